// C ABI of libscprop: system build, layout planning, and the propagate /
// fidelity / apply entry points.  See include/scprop.h for the contract.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>

#include "internal.h"
#include "trotter.h"

namespace scp {

static thread_local std::string g_err;

// Which system last wrote checkpoints into a workspace (by base pointer), and
// the stamp of that write; an adjoint without psi0 trusts the checkpoints only
// if its system's stamp is the one recorded for its workspace.
static std::mutex g_ck_mu;
static std::map<const void*, std::pair<const scp_system*, uint64_t>> g_ck_owner;
static uint64_t g_ck_next = 0;

static void ck_record(scp_system* sys, const void* ws, int S, int ce) {
  std::lock_guard<std::mutex> lk(g_ck_mu);
  sys->ck_ws = ws;
  sys->ck_S = S;
  sys->ck_ce = ce;
  sys->ck_N = sys->n_steps;
  sys->ck_gen = ++g_ck_next;
  g_ck_owner[ws] = std::make_pair((const scp_system*)sys, sys->ck_gen);
}

static void ck_clear(scp_system* sys) {
  std::lock_guard<std::mutex> lk(g_ck_mu);
  if (sys->ck_gen != 0) {
    auto it = g_ck_owner.find(sys->ck_ws);
    if (it != g_ck_owner.end() && it->second.first == sys) g_ck_owner.erase(it);
  }
  sys->ck_gen = 0;
  sys->ck_ws = nullptr;
}

// A propagate of sys into ws (with or without checkpoints) overwrites what
// another system may have left there.
static void ck_claim(const scp_system* sys, const void* ws) {
  std::lock_guard<std::mutex> lk(g_ck_mu);
  auto it = g_ck_owner.find(ws);
  if (it != g_ck_owner.end() && it->second.first != sys) g_ck_owner.erase(it);
}

static bool ck_valid(const scp_system* sys, const void* ws, int S, int ce) {
  std::lock_guard<std::mutex> lk(g_ck_mu);
  if (sys->ck_gen == 0 || sys->ck_ws != ws || sys->ck_S != S || sys->ck_ce != ce ||
      sys->ck_N != sys->n_steps)
    return false;
  auto it = g_ck_owner.find(ws);
  return it != g_ck_owner.end() && it->second.first == sys && it->second.second == sys->ck_gen;
}

void set_error(const std::string& msg) { g_err = msg; }
scp_status fail(scp_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

hipEvent_t timing_start(const scp_system* sys, hipStream_t s) {
  if (!sys->timing) return nullptr;
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  if (hipEventRecord(e, s) != hipSuccess) {
    (void)hipEventDestroy(e);
    return nullptr;
  }
  return e;
}

void timing_stop(const scp_system* sys, hipEvent_t start, int kind, hipStream_t s) {
  if (start == nullptr) return;
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess || hipEventRecord(e, s) != hipSuccess) {
    if (e) (void)hipEventDestroy(e);
    (void)hipEventDestroy(start);
    return;
  }
  sys->tev.push_back(start);
  sys->tev.push_back(e);
  sys->tkind.push_back(kind);
}

static void timing_drop(const scp_system* sys) {
  for (hipEvent_t e : sys->tev) (void)hipEventDestroy(e);
  sys->tev.clear();
  sys->tkind.clear();
}


hipError_t launch_tables_impl(int d, int nslots, int npairs, int ndrives, int ngroups, int npulse,
                              int nsteps, double h, double T, const double* frames,
                              const double2* sops, const double2* pops, const double2* dops,
                              const int* smode, const int* pmode, float2* optab, int block_q,
                              const void* drives, const double* par, float* ctab, float* dctab,
                              double* dctab64, double* ctab64, hipStream_t s);
scp_status launch_zcomp(const void* U, int64_t D, int S, int prec, int nq, const int64_t* rows,
                        const int32_t* cols, const void* target, void* block, void* tau_out,
                        double* F_out, double* phases_out, void* cot, hipStream_t s);
hipError_t launch_phase_table(int d, int NT, int NR, int RB, int thr, int row, int nsteps,
                              double h, const double* frames, const int* tmode, const int* rmode,
                              float2* ph, hipStream_t s);
size_t drive_static_size();
void pack_drive_static(void* dst, int k, int env, int npar, int par0, int group, double omega,
                       double phase, double sigma);
scp_status launch_rk4_range(const scp_system* sys, const float2* psi0, float2* psiT, float2* state,
                            float2* lo, float4* ckpt, int ce, int S, int n0, int n1, hipStream_t s);
scp_status launch_adjoint_impl(const scp_system* sys, const void* ckpt, const void* lamT,
                               void* segbuf, void* lo, void* sum, void* lamstate, double* part,
                               int ce, int nckpt, int S, hipStream_t s);

namespace {

int default_NR(int d) {
  switch (d) {
    case 2: return 4;
    case 3: return 3;
    case 4: return 2;
    case 5: return 2;
    default: return 0;
  }
}

int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// Device scratch helper freed at scope exit.
struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

scp_status validate(const scp_system_desc* ds) {
  if (!ds) return fail(SCP_EINVAL, "null descriptor");
  if (ds->n_modes < 1 || ds->n_modes > SCP_MAX_MODES) return fail(SCP_EINVAL, "n_modes out of range");
  if (ds->n_steps < 1) return fail(SCP_EINVAL, "n_steps must be >= 1");
  if (!(ds->T > 0)) return fail(SCP_EINVAL, "T must be > 0");
  if (ds->n_couplings < 0 || ds->n_drives < 0) return fail(SCP_EINVAL, "negative counts");
  if (!ds->modes) return fail(SCP_EINVAL, "null modes");
  if (ds->n_couplings > 0 && !ds->couplings) return fail(SCP_EINVAL, "null couplings");
  if (ds->n_drives > 0 && !ds->drives) return fail(SCP_EINVAL, "null drives");
  for (int m = 0; m < ds->n_modes; ++m) {
    const scp_mode_desc& M = ds->modes[m];
    if (M.trunc < 2 || M.trunc > SCP_MAX_TRUNC) return fail(SCP_EINVAL, "trunc out of range");
    if (M.kind == SCP_MODE_TRANSMON) {
      if (M.basis_dim < 3 || M.basis_dim % 2 == 0 || M.basis_dim > 95 || M.basis_dim <= M.trunc)
        return fail(SCP_EINVAL, "transmon basis_dim must be odd, > trunc and <= 95");
      if (!(M.EC > 0) || !(M.EJ > 0)) return fail(SCP_EINVAL, "transmon EC, EJ must be > 0");
    } else if (M.kind == SCP_MODE_FLUXONIUM) {
      if (M.basis_dim <= M.trunc || M.basis_dim > 96)
        return fail(SCP_EINVAL, "fluxonium basis_dim must be > trunc and <= 96");
      if (!(M.EC > 0) || !(M.EJ >= 0) || !(M.EL > 0))
        return fail(SCP_EINVAL, "fluxonium EC, EL must be > 0, EJ >= 0");
    } else if (M.kind == SCP_MODE_RAW) {
      if (!M.raw_eps || !M.raw_ops) return fail(SCP_EINVAL, "raw mode needs raw_eps and raw_ops");
    } else {
      return fail(SCP_EINVAL, "unknown mode kind");
    }
    for (int a = 0; a < M.trunc && M.has_frame; ++a)
      if (!std::isfinite(M.frame_eps[a])) return fail(SCP_EINVAL, "non-finite frame energy");
  }
  for (int e = 0; e < ds->n_couplings; ++e) {
    const scp_coupling_desc& C = ds->couplings[e];
    if (C.i < 0 || C.j < 0 || C.i >= ds->n_modes || C.j >= ds->n_modes || C.i == C.j)
      return fail(SCP_EINVAL, "coupling modes invalid");
    for (int op : {C.op_i, C.op_j})
      if (op != SCP_OP_N && op != SCP_OP_PHI) return fail(SCP_EINVAL, "coupling op invalid");
    if ((C.op_i == SCP_OP_PHI && ds->modes[C.i].kind == SCP_MODE_TRANSMON) ||
        (C.op_j == SCP_OP_PHI && ds->modes[C.j].kind == SCP_MODE_TRANSMON))
      return fail(SCP_EINVAL, "transmon has no phase operator");
    if (!std::isfinite(C.g)) return fail(SCP_EINVAL, "non-finite coupling");
  }
  for (int k = 0; k < ds->n_drives; ++k) {
    const scp_drive_desc& R = ds->drives[k];
    if (R.mode < 0 || R.mode >= ds->n_modes) return fail(SCP_EINVAL, "drive mode invalid");
    if (R.op != SCP_OP_N && R.op != SCP_OP_PHI) return fail(SCP_EINVAL, "drive op invalid");
    if (R.op == SCP_OP_PHI && ds->modes[R.mode].kind == SCP_MODE_TRANSMON)
      return fail(SCP_EINVAL, "transmon has no phase operator");
    if (R.env < SCP_ENV_GAUSS || R.env > SCP_ENV_PWC) return fail(SCP_EINVAL, "envelope invalid");
    if (R.n_par < 1 || !R.par) return fail(SCP_EINVAL, "drive needs n_par >= 1 parameters");
    if ((R.env == SCP_ENV_GAUSS || R.env == SCP_ENV_COS_RAMP || R.env == SCP_ENV_CONST) && R.n_par != 1)
      return fail(SCP_EINVAL, "this envelope takes one parameter");
    if ((R.env == SCP_ENV_GAUSS || R.env == SCP_ENV_GAUSS_BASIS) && !(R.sigma > 0))
      return fail(SCP_EINVAL, "Gaussian sigma must be > 0");
    for (int i = 0; i < R.n_par; ++i)
      if (!std::isfinite(R.par[i])) return fail(SCP_EINVAL, "non-finite pulse parameter");
  }
  return SCP_OK;
}

// Layout planning: which modes sit in registers in each layout of a stage; the
// last layout is the base one (psi, checkpoints and natural-order stores).
scp_status make_plan(scp_system* sys) {
  Plan& P = sys->plan;
  std::memset(&P, 0, sizeof(Plan));
  const int N = sys->n_modes, d = sys->d;
  int NR = default_NR(d);
  if (NR == 0) return fail(SCP_EINVAL, "the propagator supports d in {2,3,4,5}");
  NR = std::min(NR, N);
  // A step's latency is one thread's serial work.  For small d = 3 devices,
  // three register modes leave fewer than 32 threads per column; two register
  // modes give 3x more threads with a third of the work each (measured 30-40 %
  // faster on 4-6 mode rings) at the price of more layouts.
  if (d == 3 && NR == 3 && ipow(3, N - 3) < 32) NR = 2;
  const int RB = ipow(d, NR);
  const int TPC = ipow(d, N - NR);
  if (TPC > WG_THREADS)
    return fail(SCP_EINVAL, "system too large for the on-chip path (d^(N-" + std::to_string(NR) +
                                ") > 256)");
  P.d = d;
  P.N = N;
  P.NR = NR;
  P.RB = RB;
  P.TPC = TPC;
  P.NT = N - NR;
  P.CPW = std::max(1, WG_THREADS / TPC);
  P.D = (int)sys->D;
  P.nsteps = sys->n_steps;
  P.h = (float)sys->h;
  // --- slots -----------------------------------------------------------
  std::map<std::pair<int, int>, int> slot_of;
  auto slot = [&](int m, int op) {
    auto key = std::make_pair(m, op);
    auto it = slot_of.find(key);
    if (it != slot_of.end()) return it->second;
    int s = (int)sys->slot_mode.size();
    sys->slot_mode.push_back(m);
    sys->slot_op.push_back(op);
    slot_of[key] = s;
    return s;
  };
  for (auto& c : sys->coup) {
    slot(c.i, c.op_i);
    slot(c.j, c.op_j);
  }
  for (auto& r : sys->drives) slot(r.mode, r.op);
  if ((int)sys->slot_mode.size() > MAXSLOTS) return fail(SCP_EINVAL, "too many operator slots");
  // --- layouts: paths of the coupling graph ----------------------------
  std::vector<std::vector<int>> layouts;
  std::set<std::pair<int, int>> unc;
  auto key = [](int a, int b) { return std::make_pair(std::min(a, b), std::max(a, b)); };
  for (auto& c : sys->coup) unc.insert(key(c.i, c.j));
  auto in = [](const std::vector<int>& S, int m) {
    return std::find(S.begin(), S.end(), m) != S.end();
  };
  while (!unc.empty()) {
    std::pair<int, int> e{-1, -1};
    for (auto& c : sys->coup)
      if (unc.count(key(c.i, c.j))) { e = std::make_pair(c.i, c.j); break; }
    std::vector<int> S{e.first, e.second};
    unc.erase(key(e.first, e.second));
    bool grew = true;
    while ((int)S.size() < NR && grew) {
      grew = false;
      for (int side = 0; side < 2 && !grew && (int)S.size() < NR; ++side) {
        const int end = side == 0 ? S.back() : S.front();
        for (auto& c : sys->coup) {
          int other = c.i == end ? c.j : (c.j == end ? c.i : -1);
          if (other < 0 || in(S, other) || !unc.count(key(end, other))) continue;
          unc.erase(key(end, other));
          if (side == 0) S.push_back(other);
          else S.insert(S.begin(), other);
          grew = true;
          break;
        }
      }
    }
    for (int m = 0; m < N && (int)S.size() < NR; ++m)
      if (!in(S, m)) S.push_back(m);
    layouts.push_back(S);
  }
  for (int m = 0; m < N; ++m) {
    bool found = false;
    for (auto& S : layouts) found |= in(S, m);
    if (!found) {
      std::vector<int> S{m};
      for (int q = 0; q < N && (int)S.size() < NR; ++q)
        if (q != m) S.push_back(q);
      layouts.push_back(S);
    }
  }
  if ((int)layouts.size() > MAXL) return fail(SCP_EINVAL, "coupling graph needs too many layouts");
  // The last layout is the base one (psi, checkpoints, the adjoint's natural-order
  // stores).  Make it the layout whose register modes are the most significant,
  // so that its thread modes are the fastest-varying ones and consecutive lanes
  // touch consecutive elements; rotating keeps consecutive layouts adjacent.
  {
    auto weight = [&](const std::vector<int>& S) {
      long w = 0;
      for (int m : S) w += ipow(d, N - 1 - m);
      return w;
    };
    int best = (int)layouts.size() - 1;
    for (int l = 0; l < (int)layouts.size(); ++l)
      if (weight(layouts[l]) > weight(layouts[best])) best = l;
    std::rotate(layouts.begin(), layouts.begin() + best + 1, layouts.end());
  }
  const int L = (int)layouts.size();
  P.L = L;
  std::vector<int> stride(N);
  for (int m = 0; m < N; ++m) stride[m] = ipow(d, N - 1 - m);
  for (int l = 0; l < L; ++l) {
    const auto& S = layouts[l];
    for (int p = 0; p < 8; ++p) P.lmode[l][p] = p < NR ? S[p] : -1;
    for (int p = 0; p < NR; ++p) P.reg_stride[l][p] = stride[S[p]];
    for (int r = 0; r < RB; ++r) {
      int off = 0, rr = r;
      for (int p = NR - 1; p >= 0; --p) {
        off += (rr % d) * stride[S[p]];
        rr /= d;
      }
      P.reg_off[l][r] = off;
    }
    // thread modes, digit 0 = smallest stride (largest mode index)
    std::vector<int> T;
    for (int m = N - 1; m >= 0; --m)
      if (!in(S, m)) T.push_back(m);
    for (int k = 0; k < (int)T.size(); ++k) P.tstride[l][k] = stride[T[k]];
  }
  auto pos_in = [&](int l, int m) {
    auto& S = layouts[l];
    auto it = std::find(S.begin(), S.end(), m);
    return it == S.end() ? -1 : (int)(it - S.begin());
  };
  for (int m = 0; m < N; ++m) {
    P.layout_of_mode[m] = -1;
    for (int l = 0; l < L && P.layout_of_mode[m] < 0; ++l)
      if (pos_in(l, m) >= 0) {
        P.layout_of_mode[m] = l;
        P.pos_of_mode[m] = pos_in(l, m);
      }
  }
  // --- pair terms: first factor at position p, partner at p + 1 ----------
  struct Grp { int l, p, s, j; };
  std::vector<Grp> grps;
  std::vector<std::vector<cplx>> pairW;
  for (int e = 0; e < (int)sys->coup.size(); ++e) {
    const Coupling& c = sys->coup[e];
    int l = -1, p = -1;
    bool swapped = false;
    for (int q = 0; q < L && l < 0; ++q) {
      const int pi = pos_in(q, c.i), pj = pos_in(q, c.j);
      if (pi >= 0 && pj >= 0 && (pj == pi + 1 || pi == pj + 1)) {
        l = q;
        p = std::min(pi, pj);
        swapped = pj < pi;
      }
    }
    if (l < 0) return fail(SCP_EINVAL, "coupling graph not supported by the fused path");
    const int fm = swapped ? c.j : c.i, fop = swapped ? c.op_j : c.op_i;   // first factor
    const int pm = swapped ? c.i : c.j, pop = swapped ? c.op_i : c.op_j;   // partner
    const int s1 = slot(fm, fop);
    int g = -1;
    for (int q = 0; q < (int)grps.size(); ++q)
      if (grps[q].l == l && grps[q].p == p && grps[q].s == s1) g = q;
    if (g < 0) {
      g = (int)grps.size();
      if (g >= MAXPAIRS) return fail(SCP_EINVAL, "too many coupling pairs");
      grps.push_back({l, p, s1, pm});
      pairW.push_back(std::vector<cplx>(d * d, 0.0));
    }
    const cplx* Bj = sys->modes[pm].ops[pop];
    for (int i = 0; i < d * d; ++i) pairW[g][i] += c.g * Bj[i];
    if (P.pair_ncoup[g] >= 4) return fail(SCP_EINVAL, "more than 4 couplings on one mode pair");
    P.pair_pslot[g][P.pair_ncoup[g]] = slot(pm, pop);
    P.pair_coup[g][P.pair_ncoup[g]++] = e;
  }
  P.npairs = (int)grps.size();
  int MP = 1;
  for (int l = 0; l < L; ++l)
    for (int p = 0; p + 1 < NR; ++p) {
      int cnt = 0;
      for (auto& g : grps) cnt += (g.l == l && g.p == p);
      MP = std::max(MP, cnt);
    }
  if (MP > 2) return fail(SCP_EINVAL, "more than two coupling terms per mode pair and layout");
  P.MP = MP;
  if ((int)sys->slot_mode.size() + 1 > MAXSLOTS) return fail(SCP_EINVAL, "too many operator slots");
  const int zslot = (int)sys->slot_mode.size();   // zero operator slot
  const int zpair = P.npairs;                       // zero pair operator
  for (int l = 0; l < L; ++l) {
    for (int p = 0; p < 4; ++p)
      for (int m = 0; m < 2; ++m) {
        CPair& C = P.cpair[l][p][m];
        C.slot = (int32_t)zslot;
        C.pair = (int32_t)zpair;
        C.cidx = -1;
        C.mode_i = C.mode_j = -1;
        C.hsign = 1;
      }
    for (int p = 0; p < 8; ++p) {
      P.csingle[l][p].slot = (int32_t)zslot;
      P.csingle[l][p].cidx = -1;
      P.cdiag[l][p] = 16;
      P.mode_pass[l][p] = -1;
    }
  }
  {
    std::vector<int> fill((size_t)L * 4, 0);
    for (int g = 0; g < (int)grps.size(); ++g) {
      const int m = fill[grps[g].l * 4 + grps[g].p]++;
      CPair& C = P.cpair[grps[g].l][grps[g].p][m];
      C.slot = (int32_t)grps[g].s;
      C.pair = (int32_t)g;
      C.mode_i = (int32_t)sys->slot_mode[grps[g].s];
      C.mode_j = (int32_t)grps[g].j;
    }
  }
  // --- drives: attach to a pair term with the same first factor, else a single term
  std::map<int, int> group_of_slot;
  for (auto& r : sys->drives) {
    int s1 = slot(r.mode, r.op);
    if (!group_of_slot.count(s1)) {
      int g = (int)group_of_slot.size();
      group_of_slot[s1] = g;
    }
  }
  P.ngroups = (int)group_of_slot.size();
  if (P.ngroups > MAXGROUPS) return fail(SCP_EINVAL, "too many drive groups");
  for (auto& kv : group_of_slot) {
    const int s1 = kv.first, g = kv.second, m = sys->slot_mode[s1];
    bool attached = false;
    for (int l = 0; l < L && !attached; ++l)
      for (int p = 0; p + 1 < NR && !attached; ++p)
        for (int q = 0; q < MP && !attached; ++q) {
          CPair& C = P.cpair[l][p][q];
          if (C.slot == s1 && C.cidx < 0) {
            C.cidx = (int32_t)g;
            attached = true;
          }
        }
    if (!attached) {
      const int l = P.layout_of_mode[m], p = P.pos_of_mode[m];
      if (P.csingle[l][p].slot != zslot)
        return fail(SCP_EINVAL, "two drive-only operators on one mode");
      P.csingle[l][p].slot = (int32_t)s1;
      P.csingle[l][p].cidx = (int32_t)g;
      P.has_single[l] = 1;
    }
  }
  P.has_delta = 0;
  for (int a = 0; a < 8; ++a) P.delta[16][a] = 0.f;
  for (int m = 0; m < N; ++m) {
    bool nz = false;
    for (int a = 0; a < d; ++a) {
      double v = sys->modes[m].eps[a] - sys->modes[m].frame[a];
      P.delta[m][a] = (float)v;
      nz |= v != 0.0;
    }
    const int l = P.layout_of_mode[m], p = P.pos_of_mode[m];
    if (nz) {
      P.has_delta = 1;
      P.has_diag[l] = 1;
      P.cdiag[l][p] = m;
    }
    P.mode_pass[l][p] = m;
    P.has_mode_pass[l] = 1;
    for (int th = 0; th < 3; ++th)
      for (int a = 0; a < d; ++a) P.deps[m][th][a] = (float)sys->modes[m].deps[th][a];
  }
  // drives
  int par0 = 0;
  P.ndrives = (int)sys->drives.size();
  for (int k = 0; k < P.ndrives; ++k) {
    int s = slot(sys->drives[k].mode, sys->drives[k].op);
    P.drives[k].slot = (int32_t)s;
    P.drives[k].cidx = (int32_t)group_of_slot[s];
    P.drives[k].par0 = (int32_t)par0;
    P.drives[k].npar = (int32_t)sys->drives[k].par.size();
    par0 += (int)sys->drives[k].par.size();
  }
  P.npulse = par0;
  if (P.npulse > MAXPULSE) return fail(SCP_EINVAL, "too many pulse parameters");
  // drives of each mode (adjoint mode pass), each slot's coefficient counted once
  {
    int q = 0;
    for (int m = 0; m < N; ++m) {
      P.mdrv_off[m] = q;
      for (int k = 0; k < P.ndrives; ++k) {
        if (sys->drives[k].mode != m) continue;
        bool first = true;
        for (int k2 = 0; k2 < k; ++k2) first &= P.drives[k2].slot != P.drives[k].slot;
        P.mdrv[q] = (int32_t)k;
        P.mdrv_first[q] = first ? 1 : 0;
        ++q;
      }
    }
    for (int m = N; m <= 16; ++m) P.mdrv_off[m] = q;
  }
  P.nslots = (int)sys->slot_mode.size() + 1;   // + the zero slot
  for (int s = 0; s < P.nslots - 1; ++s) {
    P.slot_mode[s] = sys->slot_mode[s];
    P.slot_op[s] = sys->slot_op[s];
  }
  P.ncoup = (int)sys->coup.size();
  for (int e = 0; e < P.ncoup; ++e) {
    P.coup_g[e] = (float)sys->coup[e].g;
    P.coup_slot_i[e] = slot(sys->coup[e].i, sys->coup[e].op_i);
    P.coup_slot_j[e] = slot(sys->coup[e].j, sys->coup[e].op_j);
  }
  P.nacc = P.npulse + 3 * N + P.ncoup;
  P.off_pair = P.nslots * d * d;
  P.off_dslot = (P.nslots + P.npairs + 1) * d * d;
  P.block_q = (P.nslots + P.npairs + 1 + 3 * P.nslots) * d * d;
  // LDS per workgroup: three column-sized regions per column (stepper: the
  // stage input and two regions for the moves of k; adjoint: kb, y and the
  // pass of yb), plus the adjoint's FP64 accumulators (4 waves max).
  {
    const long budget = 163840 - 4L * 8 * std::max(1, P.nacc);
    const long per_col = 3L * 8 * P.D;
    const int cpw_lds = (int)(budget / per_col);
    if (cpw_lds < 1) return fail(SCP_EINVAL, "system too large for the on-chip path (LDS)");
    P.CPW = std::min(P.CPW, cpw_lds);
  }
  int threads = P.CPW * TPC;
  P.WG = ((threads + 63) / 64) * 64;
  // host copy of pair W for the table kernel
  sys->pairW_host.clear();
  sys->pair_mode_host.clear();
  for (int p = 0; p < P.npairs; ++p) {
    for (auto v : pairW[p]) sys->pairW_host.push_back(v);
    sys->pair_mode_host.push_back(grps[p].j);
  }
  for (int i = 0; i < d * d; ++i) sys->pairW_host.push_back(0.0);   // zero pair operator
  sys->pair_mode_host.push_back(0);
  // real frame: every operator real (kind 1) or i times real (kind 2), zero
  // operators both (3); a slot's derivatives share its kind, the partner
  // operators of a pair term share the first factor's kind (the term is then
  // +-1 times a real one), and drives sit on real operators
  auto kind_of = [&](const cplx* o) {
    bool re0 = true, im0 = true;
    for (int i = 0; i < d * d; ++i) {
      re0 = re0 && o[i].real() == 0.0;
      im0 = im0 && o[i].imag() == 0.0;
    }
    return (im0 ? 1 : 0) | (re0 ? 2 : 0);
  };
  const int nsl = (int)sys->slot_mode.size();
  std::vector<int> skind(nsl + 1, 3);   // + the zero slot
  for (int s = 0; s < nsl; ++s) {
    const ModeData& M = sys->modes[sys->slot_mode[s]];
    int k = kind_of(M.ops[sys->slot_op[s]]);
    for (int th = 0; th < 3; ++th) k &= kind_of(M.dops[th][sys->slot_op[s]]);
    skind[s] = k;
  }
  bool real = true;
  std::vector<int> pkind(P.npairs + 1, 3);
  for (int g = 0; g < P.npairs; ++g) {
    int k = skind[grps[g].s];
    for (int q = 0; q < P.pair_ncoup[g]; ++q) k &= skind[P.pair_pslot[g][q]];
    pkind[g] = k;
    real = real && k != 0;
  }
  for (int k = 0; k < P.ndrives; ++k) real = real && (skind[P.drives[k].slot] & 1) != 0;
  P.real_frame = real ? 1 : 0;
  sys->slot_imag.assign(nsl + 1, 0);
  sys->pair_imag.assign(P.npairs + 1, 0);
  if (real) {
    for (int s = 0; s <= nsl; ++s) sys->slot_imag[s] = skind[s] == 2;
    for (int g = 0; g < P.npairs; ++g) sys->pair_imag[g] = pkind[g] == 2;
    for (int l = 0; l < P.L; ++l)
      for (int p = 0; p < 4; ++p)
        for (int m = 0; m < 2; ++m) {
          CPair& C = P.cpair[l][p][m];
          C.hsign = (C.pair < P.npairs && sys->pair_imag[C.pair]) ? -1 : 1;
        }
  }
  P.ph_thr = (P.RB + 7) / 8 * 8;
  P.ph_row = (P.ph_thr + P.NT * d + 7) / 8 * 8;
  return SCP_OK;
}

scp_status build_tables(scp_system* sys, hipStream_t st) {
  const Plan& P = sys->plan;
  const int d = sys->d, dd = d * d, N = sys->n_modes;
  const int ns = P.nslots, np1 = P.npairs + 1;   // both include a trailing zero operator
  std::vector<double> frames((size_t)N * 8, 0.0);
  for (int m = 0; m < N; ++m)
    for (int a = 0; a < d; ++a) frames[m * 8 + a] = sys->modes[m].frame[a];
  std::vector<double2> sops((size_t)ns * dd, make_double2(0, 0)), pops((size_t)np1 * dd, make_double2(0, 0)),
      dops((size_t)ns * 3 * dd, make_double2(0, 0));
  for (int s = 0; s < ns - 1; ++s) {
    const ModeData& M = sys->modes[P.slot_mode[s]];
    for (int i = 0; i < dd; ++i) {
      cplx v = M.ops[P.slot_op[s]][i];
      sops[s * dd + i] = make_double2(v.real(), v.imag());
      for (int th = 0; th < 3; ++th) {
        cplx dv = M.dops[th][P.slot_op[s]][i];
        dops[(s * 3 + th) * dd + i] = make_double2(dv.real(), dv.imag());
      }
    }
  }
  for (int p = 0; p < np1; ++p)
    for (int i = 0; i < dd; ++i) {
      cplx v = sys->pairW_host[p * dd + i];
      pops[p * dd + i] = make_double2(v.real(), v.imag());
    }
  std::vector<int> smode(ns, 0), pmode(np1, 0);
  for (int s = 0; s < ns - 1; ++s) smode[s] = P.slot_mode[s];
  for (int p = 0; p < np1; ++p) pmode[p] = sys->pair_mode_host[p];
  // drives
  std::vector<char> dstat(drive_static_size() * std::max<size_t>(1, sys->drives.size()));
  std::vector<double> par;
  for (int k = 0; k < (int)sys->drives.size(); ++k) {
    const Drive& R = sys->drives[k];
    pack_drive_static(dstat.data(), k, R.env, (int)R.par.size(), (int)par.size(),
                      P.drives[k].cidx, R.omega, R.phase, R.sigma);
    for (double v : R.par) par.push_back(v);
  }
  if (par.empty()) par.push_back(0.0);
  // temporary device copies
  DevBuf bf, bs, bp, bd, bsm, bpm, bdr, bpar;
  HIPCHK(hipMalloc(&bf.p, frames.size() * sizeof(double)));
  HIPCHK(hipMalloc(&bs.p, sops.size() * sizeof(double2)));
  HIPCHK(hipMalloc(&bp.p, pops.size() * sizeof(double2)));
  HIPCHK(hipMalloc(&bd.p, dops.size() * sizeof(double2)));
  HIPCHK(hipMalloc(&bsm.p, smode.size() * sizeof(int)));
  HIPCHK(hipMalloc(&bpm.p, pmode.size() * sizeof(int)));
  HIPCHK(hipMalloc(&bdr.p, dstat.size()));
  HIPCHK(hipMalloc(&bpar.p, par.size() * sizeof(double)));
  HIPCHK(hipMemcpyAsync(bf.p, frames.data(), frames.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(bs.p, sops.data(), sops.size() * sizeof(double2), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(bp.p, pops.data(), pops.size() * sizeof(double2), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(bd.p, dops.data(), dops.size() * sizeof(double2), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(bsm.p, smode.data(), smode.size() * sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(bpm.p, pmode.data(), pmode.size() * sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(bdr.p, dstat.data(), dstat.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(bpar.p, par.data(), par.size() * sizeof(double), hipMemcpyHostToDevice, st));
  const size_t nq = 2 * (size_t)sys->n_steps + 1;
  HIPCHK(hipMalloc(&sys->d_ops, nq * P.block_q * sizeof(float2)));
  const size_t np3 = 3 * (size_t)sys->n_steps;
  HIPCHK(hipMalloc(&sys->d_ctab, np3 * std::max(1, P.ngroups) * sizeof(float)));
  HIPCHK(hipMalloc(&sys->d_dctab, np3 * std::max(1, P.npulse) * sizeof(float)));
  HIPCHK(hipMalloc(&sys->d_dctab64, np3 * std::max(1, P.npulse) * sizeof(double)));
  HIPCHK(hipMalloc(&sys->d_ctab64, np3 * std::max<size_t>(1, sys->drives.size()) * sizeof(double)));
  HIPCHK(launch_tables_impl(d, ns, np1, (int)sys->drives.size(), P.ngroups, P.npulse,
                            sys->n_steps, sys->h, sys->T, (const double*)bf.p,
                            (const double2*)bs.p, (const double2*)bp.p, (const double2*)bd.p,
                            (const int*)bsm.p, (const int*)bpm.p, sys->d_ops, P.block_q, bdr.p,
                            (const double*)bpar.p, sys->d_ctab, sys->d_dctab, sys->d_dctab64,
                            sys->d_ctab64, st));
  DevBuf bmodes;
  sys->real_ok = P.real_frame != 0;
  if (P.real_frame) {
    // modes at the thread positions (by natural stride) and at the register
    // positions of the base layout
    const int base = P.L - 1;
    std::vector<int> modes(P.NT + P.NR, 0);
    for (int k = 0; k < P.NT; ++k)
      for (int m = 0; m < N; ++m) {
        int64_t st_m = 1;
        for (int q = m + 1; q < N; ++q) st_m *= d;
        if (st_m == P.tstride[base][k]) modes[k] = m;
      }
    for (int p = 0; p < P.NR; ++p) modes[P.NT + p] = P.lmode[base][p];
    HIPCHK(hipMalloc(&bmodes.p, modes.size() * sizeof(int)));
    HIPCHK(hipMemcpyAsync(bmodes.p, modes.data(), modes.size() * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMalloc(&sys->d_ph, nq * P.ph_row * sizeof(float2)));
    // the operators at t = 0 (the table's block 0 rounds them the same way)
    // (kind 2: the imaginary parts; a pair term of kind 2 is i^2 = -1 times the
    // product of the real parts, folded into the pair operator's sign)
    std::vector<float> rops(P.block_q, 0.f);
    auto put = [&](int at, double x) { rops[at] = (float)x; };
    for (int s = 0; s < ns; ++s)
      for (int i = 0; i < dd; ++i) {
        const bool im = sys->slot_imag[s] != 0;
        put(s * dd + i, im ? sops[s * dd + i].y : sops[s * dd + i].x);
        for (int th = 0; th < 3; ++th) {
          const double2 v = dops[(s * 3 + th) * dd + i];
          put(P.off_dslot + (s * 3 + th) * dd + i, im ? v.y : v.x);
        }
      }
    for (int p = 0; p < np1; ++p)
      for (int i = 0; i < dd; ++i)
        put(P.off_pair + p * dd + i, sys->pair_imag[p] ? -pops[p * dd + i].y : pops[p * dd + i].x);
    HIPCHK(hipMalloc(&sys->d_rops, rops.size() * sizeof(float)));
    HIPCHK(hipMemcpyAsync(sys->d_rops, rops.data(), rops.size() * sizeof(float), hipMemcpyHostToDevice, st));
    HIPCHK(launch_phase_table(d, P.NT, P.NR, P.RB, P.ph_thr, P.ph_row, sys->n_steps, sys->h,
                              (const double*)bf.p, (const int*)bmodes.p,
                              (const int*)bmodes.p + P.NT, sys->d_ph, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  return SCP_OK;
}

// A mode truncated to dm < d levels is carried at the system's d levels.  The
// extra levels have no operator element to or from any level (zero rows and
// columns in n, phi and their derivatives), so no amplitude ever enters them
// and the dm levels evolve exactly as in the product space of the modes' own
// truncations.  Their energies continue the top level spacing (distinct; in
// a spectrum they are uncoupled states of their own).
void pad_mode(ModeData& md, int d) {
  const int dm = md.d;
  if (dm >= d) return;
  auto pad = [&](cplx* a) {
    cplx t[SCP_MAX_TRUNC * SCP_MAX_TRUNC];
    for (int i = 0; i < d * d; ++i) t[i] = cplx(0.0, 0.0);
    for (int r = 0; r < dm; ++r)
      for (int c = 0; c < dm; ++c) t[r * d + c] = a[r * dm + c];
    std::copy(t, t + d * d, a);
  };
  for (int o = 0; o < 2; ++o) pad(md.ops[o]);
  for (int p = 0; p < 3; ++p) {
    for (int o = 0; o < 2; ++o) pad(md.dops[p][o]);
    for (int a = dm; a < d; ++a) md.deps[p][a] = 0.0;
  }
  const double gap = md.eps[dm - 1] - md.eps[dm - 2];
  for (int a = dm; a < d; ++a) md.eps[a] = md.eps[dm - 1] + (a - dm + 1) * (gap > 0 ? gap : 1.0);
  md.d = d;
}

scp_status build(const scp_system_desc* ds, hipStream_t st, scp_system* sys) {
  scp_status v = validate(ds);
  if (v != SCP_OK) return v;
  HIPCHK(hipGetDevice(&sys->device));
  const int N = ds->n_modes;
  sys->n_modes = N;
  // modes of different truncations run at the largest, the others padded
  sys->d = 0;
  for (int m = 0; m < N; ++m) sys->d = std::max(sys->d, (int)ds->modes[m].trunc);
  sys->n_steps = ds->n_steps;
  sys->T = ds->T;
  sys->h = ds->T / ds->n_steps;
  sys->D = 1;
  for (int m = 0; m < N; ++m) sys->D *= sys->d;
  sys->modes.resize(N);
  // host basis matrices
  std::vector<int> eig_modes;
  for (int m = 0; m < N; ++m) {
    const scp_mode_desc& M = ds->modes[m];
    ModeData& md = sys->modes[m];
    md.kind = M.kind;
    md.d = M.trunc;
    md.K = M.basis_dim;
    md.EC = M.EC;
    md.EJ = M.EJ;
    md.EL = M.EL;
    md.ng = M.ng;
    md.phiext = M.phiext;
    if (M.kind == SCP_MODE_TRANSMON) {
      build_transmon(md);
      eig_modes.push_back(m);
    } else if (M.kind == SCP_MODE_FLUXONIUM) {
      build_fluxonium(md);
      eig_modes.push_back(m);
    } else {
      const int d = M.trunc;
      md.has_phi = true;
      for (int a = 0; a < d; ++a) md.eps[a] = M.raw_eps[a];
      for (int o = 0; o < 2; ++o)
        for (int i = 0; i < d * d; ++i)
          md.ops[o][i] = cplx(M.raw_ops[(o * d * d + i) * 2], M.raw_ops[(o * d * d + i) * 2 + 1]);
      for (int p = 0; p < 3; ++p) {
        for (int a = 0; a < d; ++a) md.deps[p][a] = 0.0;
        for (int o = 0; o < 2; ++o)
          for (int i = 0; i < d * d; ++i) md.dops[p][o][i] = 0.0;
      }
    }
  }
  // FP64 eigensolves on the device, one workgroup per mode
  if (!eig_modes.empty()) {
    std::vector<int> Ks;
    std::vector<int64_t> offs;
    int64_t tot = 0;
    for (int m : eig_modes) {
      Ks.push_back(sys->modes[m].K);
      offs.push_back(tot);
      tot += (int64_t)sys->modes[m].K * sys->modes[m].K;
    }
    std::vector<double> A(tot);
    for (size_t i = 0; i < eig_modes.size(); ++i) {
      const ModeData& md = sys->modes[eig_modes[i]];
      std::copy(md.H.begin(), md.H.end(), A.begin() + offs[i]);
    }
    DevBuf bA, bV, bw, bK, bo;
    HIPCHK(hipMalloc(&bA.p, tot * sizeof(double)));
    HIPCHK(hipMalloc(&bV.p, tot * sizeof(double)));
    HIPCHK(hipMalloc(&bw.p, tot * sizeof(double)));
    HIPCHK(hipMalloc(&bK.p, Ks.size() * sizeof(int)));
    HIPCHK(hipMalloc(&bo.p, offs.size() * sizeof(int64_t)));
    HIPCHK(hipMemcpyAsync(bA.p, A.data(), tot * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(bK.p, Ks.data(), Ks.size() * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(bo.p, offs.data(), offs.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
    HIPCHK(launch_jacobi((double*)bA.p, (double*)bV.p, (double*)bw.p, (const int*)bK.p,
                         (const int64_t*)bo.p, (int)eig_modes.size(), st));
    std::vector<double> V(tot), w(tot);
    HIPCHK(hipMemcpyAsync(V.data(), bV.p, tot * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(w.data(), bw.p, tot * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (size_t i = 0; i < eig_modes.size(); ++i) {
      ModeData& md = sys->modes[eig_modes[i]];
      const int K = md.K;
      md.V.assign(V.begin() + offs[i], V.begin() + offs[i] + (int64_t)K * K);
      md.w.assign(w.begin() + offs[i], w.begin() + offs[i] + K);
      scp_status s = finish_mode(md);
      if (s != SCP_OK) return s;
    }
  }
  for (int m = 0; m < N; ++m) pad_mode(sys->modes[m], sys->d);
  // frames (a padded level's frame is its energy), couplings, drives
  for (int m = 0; m < N; ++m) {
    const scp_mode_desc& M = ds->modes[m];
    for (int a = 0; a < sys->d; ++a)
      sys->modes[m].frame[a] = M.has_frame && a < M.trunc ? M.frame_eps[a] : sys->modes[m].eps[a];
  }
  for (int e = 0; e < ds->n_couplings; ++e) {
    const scp_coupling_desc& C = ds->couplings[e];
    sys->coup.push_back({C.i, C.j, C.op_i, C.op_j, C.g});
  }
  for (int k = 0; k < ds->n_drives; ++k) {
    const scp_drive_desc& R = ds->drives[k];
    Drive dr;
    dr.mode = R.mode;
    dr.op = R.op;
    dr.env = R.env;
    dr.phase = R.phase;
    dr.sigma = R.sigma;
    const double* f = sys->modes[R.mode].frame;
    dr.omega = R.has_omega ? R.omega_d : (f[1] - f[0]);
    dr.par.assign(R.par, R.par + R.n_par);
    sys->drives.push_back(dr);
    sys->n_pulse += R.n_par;
  }
  sys->n_params = sys->n_pulse + 3 * N + (int)sys->coup.size();
  scp_status s = make_plan(sys);
  if (s != SCP_OK) return s;
  HIPCHK(hipMalloc((void**)&sys->d_plan, sizeof(Plan)));
  HIPCHK(hipMemcpyAsync(sys->d_plan, &sys->plan, sizeof(Plan), hipMemcpyHostToDevice, st));
  return build_tables(sys, st);
}

// Workspace layout (bytes)
struct WsLayout {
  size_t lo = 0, ckpt = 0, seg = 0, part = 0, lam = 0, lamstate = 0, total = 0;
  int nckpt = 0, ce = 0, nwg = 0;
  bool gather = false;        // a forward-only FP32 solve on the gather engine (workspace from 0)
  bool gather_grad = false;   // checkpoints / adjoint on the gather engine (its own layout)
};

// Which engine runs an FP32 solve: the system's choice, else (automatic) the
// gather engine when the register-layout stepper would leave most of the chip
// idle.  allow_gather = false keeps the register-layout engine.
WsLayout ws_layout(const scp_system* sys, const scp_solve_opts* o, int with_grad,
                   bool allow_gather = true) {
  WsLayout w;
  const int N = sys->n_steps;
  w.ce = o->ckpt_every > 0 ? o->ckpt_every : (int)std::ceil(std::sqrt((double)N));
  w.nckpt = (N + w.ce - 1) / w.ce;
  const size_t S = (size_t)o->n_cols, D = (size_t)sys->D;
  size_t off = 0;
  auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const int engine = allow_gather ? sys->engine : 1;
  bool want = false;
  if (o->precision == 0 && engine != 1)
    want = engine == 2 ? gather_supported(sys) : gather_preferred(sys, (int)S);
  if (want && (o->with_ckpt || with_grad)) {
    want = gather_grad_check(sys) == SCP_OK;
    if (!want) set_error("");
  }
  if (want && !o->with_ckpt && !with_grad) {
    w.gather = true;
    off = gather_workspace_bytes(sys);
  } else if (want) {
    w.gather_grad = true;
    off = gather_grad_workspace_bytes(sys, (int)S, w.ce, with_grad != 0);
  } else if (o->precision == 0) {
    w.lo = off;
    off = align(off + S * D * sizeof(float2));
    if (o->with_ckpt || with_grad) {
      w.ckpt = off;
      off = align(off + (size_t)w.nckpt * S * D * sizeof(float4));
    }
    if (with_grad) {
      w.nwg = (int)((S + sys->plan.CPW - 1) / sys->plan.CPW);
      w.seg = off;
      off = align(off + (size_t)w.ce * 4 * S * D * sizeof(float2));
      w.lam = off;
      off = align(off + S * D * sizeof(float2));
      w.lamstate = off;
      off = align(off + S * D * sizeof(float2));
      w.part = off;
      off = align(off + (size_t)w.nwg * 4 * std::max(1, sys->plan.nacc) * sizeof(double));
    }
  } else {
    off = align(4 * S * D * sizeof(double2));
  }
  w.total = std::max<size_t>(off, 256);
  return w;
}

}  // namespace

scp_status finish_adjoint(scp_system* sys, const WsLayout& w, char* ws, const void* cotangent,
                          double* grad_out, int S, hipStream_t st);

}  // namespace scp

using namespace scp;

extern "C" {

const char* scp_last_error(void) { return g_err.c_str(); }

scp_status scp_build_system(const scp_system_desc* desc, void* stream, scp_system** out) {
  g_err.clear();
  if (!out) return fail(SCP_EINVAL, "null out");
  *out = nullptr;
  scp_system* sys = new (std::nothrow) scp_system();
  if (!sys) return fail(SCP_ENOMEM, "host allocation");
  scp_status s = build(desc, (hipStream_t)stream, sys);
  if (s != SCP_OK) {
    scp_destroy(sys);
    return s;
  }
  *out = sys;
  return SCP_OK;
}

scp_status scp_system_info(const scp_system* sys, int64_t* D, int32_t* n_params, int32_t* n_modes,
                           int32_t* dims) {
  if (!sys) return fail(SCP_EINVAL, "null system");
  if (D) *D = sys->D;
  if (n_params) *n_params = sys->n_params;
  if (n_modes) *n_modes = sys->n_modes;
  if (dims)
    for (int m = 0; m < sys->n_modes; ++m) dims[m] = sys->d;
  return SCP_OK;
}

scp_status scp_system_mode(const scp_system* sys, int32_t mode, double* eps, double* frame,
                           double* ops) {
  if (!sys || mode < 0 || mode >= sys->n_modes) return fail(SCP_EINVAL, "bad mode");
  const ModeData& m = sys->modes[mode];
  const int d = sys->d;
  for (int a = 0; a < d; ++a) {
    if (eps) eps[a] = m.eps[a];
    if (frame) frame[a] = m.frame[a];
  }
  if (ops)
    for (int o = 0; o < 2; ++o)
      for (int i = 0; i < d * d; ++i) {
        ops[(o * d * d + i) * 2] = m.ops[o][i].real();
        ops[(o * d * d + i) * 2 + 1] = m.ops[o][i].imag();
      }
  return SCP_OK;
}

scp_status scp_system_carriers(const scp_system* sys, double* omega) {
  if (!sys || !omega) return fail(SCP_EINVAL, "null argument");
  for (size_t k = 0; k < sys->drives.size(); ++k) omega[k] = sys->drives[k].omega;
  return SCP_OK;
}

scp_status scp_system_frame(const scp_system* sys, int32_t* real_frame) {
  if (!sys || !real_frame) return fail(SCP_EINVAL, "null argument");
  *real_frame = sys->plan.real_frame;
  return SCP_OK;
}

scp_status scp_system_set_frame(scp_system* sys, int32_t real_frame) {
  g_err.clear();
  if (!sys) return fail(SCP_EINVAL, "null argument");
  if (real_frame != 0 && real_frame != 1) return fail(SCP_EINVAL, "real_frame must be 0 or 1");
  if (real_frame && !sys->real_ok) return fail(SCP_EINVAL, "the system has complex operators");
  if (sys->plan.real_frame != real_frame) ck_clear(sys);   // checkpoints of the other evaluation
  sys->plan.real_frame = real_frame;
  HIPCHK(hipMemcpy(&sys->d_plan->real_frame, &sys->plan.real_frame, sizeof(int32_t),
                   hipMemcpyHostToDevice));
  return SCP_OK;
}

scp_status scp_system_set_engine(scp_system* sys, int32_t engine) {
  g_err.clear();
  if (!sys) return fail(SCP_EINVAL, "null argument");
  if (engine < 0 || engine > 2) return fail(SCP_EINVAL, "engine must be 0, 1 or 2");
  if (engine == 2 && !gather_supported(sys))
    return fail(SCP_EINVAL, "the gather engine has no stepper for this device (64 <= D <= 4096, "
                            "at most 10 modes, tables within the LDS)");
  if (sys->engine != engine) ck_clear(sys);   // checkpoints of the other engine's layout
  sys->engine = engine;
  return SCP_OK;
}

scp_status scp_solve_engine(const scp_system* sys, const scp_solve_opts* opts, int32_t with_grad,
                            int32_t* engine) {
  g_err.clear();
  if (!sys || !opts || !engine) return fail(SCP_EINVAL, "null argument");
  if (opts->n_cols < 1) return fail(SCP_EINVAL, "n_cols must be >= 1");
  if (opts->precision != 0) {
    *engine = 0;
    return SCP_OK;
  }
  const WsLayout w = ws_layout(sys, opts, with_grad);
  *engine = (w.gather || w.gather_grad) ? 2 : 1;
  return SCP_OK;
}

scp_status scp_system_set_timing(scp_system* sys, int32_t enable) {
  g_err.clear();
  if (!sys || (enable != 0 && enable != 1)) return fail(SCP_EINVAL, "bad argument");
  sys->timing = enable != 0;
  if (!sys->timing) timing_drop(sys);
  return SCP_OK;
}

scp_status scp_system_kernel_times(scp_system* sys, double* ms_out, int32_t* counts) {
  g_err.clear();
  if (!sys || !ms_out || !counts) return fail(SCP_EINVAL, "null argument");
  for (int k = 0; k < 3; ++k) {
    ms_out[k] = 0.0;
    counts[k] = 0;
  }
  for (size_t i = 0; i < sys->tkind.size(); ++i) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(sys->tev[2 * i + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, sys->tev[2 * i], sys->tev[2 * i + 1]);
    if (e != hipSuccess) {
      timing_drop(sys);
      return fail(SCP_EHIP, std::string("kernel timing: ") + hipGetErrorString(e));
    }
    ms_out[sys->tkind[i]] += ms;
    counts[sys->tkind[i]] += 1;
  }
  timing_drop(sys);
  return SCP_OK;
}

scp_status scp_workspace_size(const scp_system* sys, const scp_solve_opts* opts, int32_t with_grad,
                              size_t* bytes) {
  if (!sys || !opts || !bytes) return fail(SCP_EINVAL, "null argument");
  if (opts->n_cols < 1) return fail(SCP_EINVAL, "n_cols must be >= 1");
  *bytes = ws_layout(sys, opts, with_grad).total;
  return SCP_OK;
}

scp_status scp_apply_generator(const scp_system* sys, int32_t step, int32_t stage, const void* y,
                               void* out, int32_t n_cols, void* stream) {
  g_err.clear();
  if (!sys || !y || !out) return fail(SCP_EINVAL, "null argument");
  if (step < 0 || step >= sys->n_steps || stage < 0 || stage > 3 || n_cols < 1)
    return fail(SCP_EINVAL, "step/stage/n_cols out of range");
  return launch_apply(sys, step, stage, (const float2*)y, (float2*)out, n_cols, (hipStream_t)stream);
}

scp_status scp_propagate(scp_system* sys, const scp_solve_opts* opts, void* workspace,
                         const void* psi0, void* psiT, void* stream) {
  g_err.clear();
  if (!sys || !opts || !psi0 || !psiT) return fail(SCP_EINVAL, "null argument");
  if (opts->n_cols < 1) return fail(SCP_EINVAL, "n_cols must be >= 1");
  if (opts->precision != 0 && opts->precision != 1) return fail(SCP_EINVAL, "precision must be 0 or 1");
  if (opts->ckpt_every < 0) return fail(SCP_EINVAL, "ckpt_every must be >= 0");
  WsLayout w = ws_layout(sys, opts, 0);
  if (!workspace) return fail(SCP_EINVAL, "a workspace is needed (scp_workspace_size)");
  if (opts->workspace_bytes < w.total)
    return fail(SCP_EINVAL, "workspace_bytes " + std::to_string(opts->workspace_bytes) +
                                " below the " + std::to_string(w.total) + " these opts need");
  hipStream_t st = (hipStream_t)stream;
  ck_claim(sys, workspace);
  if (opts->precision == 1) {
    ck_clear(sys);
    return launch_plain64(sys, (const double2*)psi0, (double2*)psiT, workspace, opts->n_cols, st);
  }
  if (w.gather) {
    ck_clear(sys);
    return launch_gather_forward(sys, opts->n_cols, workspace, opts->workspace_bytes,
                                 (const float2*)psi0, (float2*)psiT, st);
  }
  if (w.gather_grad) {
    ck_clear(sys);
    scp_status s = launch_gather_ckpt_forward(sys, opts->n_cols, w.ce, workspace,
                                              opts->workspace_bytes, (const float2*)psi0,
                                              (float2*)psiT, st);
    if (s == SCP_OK) ck_record(sys, workspace, opts->n_cols, w.ce);
    return s;
  }
  float4* ck = opts->with_ckpt ? (float4*)((char*)workspace + w.ckpt) : nullptr;
  ck_clear(sys);
  scp_status s = launch_rk4(sys, (const float2*)psi0, (float2*)psiT,
                            (float2*)((char*)workspace + w.lo), ck, w.ce, opts->n_cols, st);
  if (s == SCP_OK && ck != nullptr) ck_record(sys, workspace, opts->n_cols, w.ce);
  return s;
}

scp_status scp_trotter_workspace_size(const scp_system* sys, int32_t order, size_t* bytes) {
  g_err.clear();
  if (!sys || !bytes) return fail(SCP_EINVAL, "null argument");
  scp_status st = trotter_check(sys, order);
  if (st != SCP_OK) return st;
  *bytes = trotter_workspace_bytes(sys, order);
  return SCP_OK;
}

scp_status scp_propagate_trotter(scp_system* sys, int32_t order, int32_t n_cols, void* workspace,
                                 const void* psi0, void* psiT, void* stream) {
  g_err.clear();
  if (!sys || !workspace || !psi0 || !psiT) return fail(SCP_EINVAL, "null argument");
  if (n_cols < 1) return fail(SCP_EINVAL, "n_cols must be >= 1");
  return launch_trotter(sys, order, n_cols, workspace, (const double2*)psi0, (double2*)psiT,
                        (hipStream_t)stream);
}

scp_status scp_lindblad_workspace_size(const scp_system* sys, size_t* bytes) {
  g_err.clear();
  if (!sys || !bytes) return fail(SCP_EINVAL, "null argument");
  const scp_status st = lindblad_check(sys);
  if (st != SCP_OK) return st;
  *bytes = lindblad_workspace_bytes(sys);
  return SCP_OK;
}

scp_status scp_propagate_lindblad(scp_system* sys, const double* gamma1, const double* gammaphi,
                                  int32_t n_cols, void* workspace, size_t workspace_bytes,
                                  const void* rho0, void* rhoT, void* stream) {
  g_err.clear();
  if (!sys || !workspace || !rho0 || !rhoT) return fail(SCP_EINVAL, "null argument");
  if (n_cols < 1) return fail(SCP_EINVAL, "n_cols must be >= 1");
  if (rho0 == rhoT) return fail(SCP_EINVAL, "rhoT must not alias rho0");
  return launch_lindblad(sys, gamma1, gammaphi, n_cols, workspace, workspace_bytes,
                         (const float2*)rho0, (float2*)rhoT, (hipStream_t)stream);
}

scp_status scp_lindblad_adjoint_workspace_size(const scp_system* sys, int32_t n_cols,
                                               size_t* bytes) {
  g_err.clear();
  if (!sys || !bytes) return fail(SCP_EINVAL, "null argument");
  if (n_cols < 1) return fail(SCP_EINVAL, "n_cols must be >= 1");
  return lindblad_adjoint_workspace_bytes(sys, n_cols, bytes);
}

scp_status scp_lindblad_adjoint(scp_system* sys, const double* gamma1, const double* gammaphi,
                                int32_t n_cols, void* workspace, size_t workspace_bytes,
                                const void* rho0, const void* cotangent, double* grad_out,
                                void* stream) {
  g_err.clear();
  if (!sys || !workspace || !rho0 || !cotangent || !grad_out) return fail(SCP_EINVAL, "null argument");
  if (n_cols < 1) return fail(SCP_EINVAL, "n_cols must be >= 1");
  return launch_lindblad_adjoint(sys, gamma1, gammaphi, n_cols, workspace, workspace_bytes,
                                 (const float2*)rho0, (const float2*)cotangent, grad_out,
                                 (hipStream_t)stream);
}

scp_status scp_fidelity_channel(const void* rhoT, int64_t D, int32_t d_c, const int64_t* comp_rows,
                                const void* target, void* overlap_out, void* cotangent,
                                double* F_out, void* stream) {
  g_err.clear();
  if (!rhoT || !comp_rows || !target || !overlap_out) return fail(SCP_EINVAL, "null argument");
  if (D < 1 || d_c < 1 || d_c > D) return fail(SCP_EINVAL, "need 1 <= d_c <= D");
  hipStream_t st = (hipStream_t)stream;
  scp_status s = launch_fidelity_channel(rhoT, D, d_c, comp_rows, target, overlap_out, cotangent, st);
  if (s != SCP_OK || !F_out) return s;
  double ov[2];
  HIPCHK(hipMemcpyAsync(ov, overlap_out, sizeof(ov), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (!std::isfinite(ov[0]) || !std::isfinite(ov[1])) return fail(SCP_ENONFINITE, "non-finite overlap");
  *F_out = (ov[0] + d_c) / ((double)d_c * (d_c + 1.0));
  return SCP_OK;
}

scp_status scp_trotter_adjoint_workspace_size(const scp_system* sys, int32_t order, int32_t n_cols,
                                              size_t* bytes) {
  g_err.clear();
  if (!sys || !bytes) return fail(SCP_EINVAL, "null argument");
  if (n_cols < 1) return fail(SCP_EINVAL, "n_cols must be >= 1");
  scp_status st = trotter_adjoint_check(sys, order);
  if (st != SCP_OK) return st;
  *bytes = trotter_adjoint_workspace_bytes(sys, order, n_cols);
  return SCP_OK;
}

scp_status scp_propagate_trotter_adjoint(scp_system* sys, int32_t order, int32_t n_cols,
                                         void* workspace, size_t workspace_bytes, const void* psi0,
                                         const void* cotangent, double* grad_out, void* stream) {
  g_err.clear();
  if (!sys || !workspace || !psi0 || !cotangent || !grad_out) return fail(SCP_EINVAL, "null argument");
  if (n_cols < 1) return fail(SCP_EINVAL, "n_cols must be >= 1");
  scp_status st = trotter_adjoint_check(sys, order);
  if (st != SCP_OK) return st;
  const size_t need = trotter_adjoint_workspace_bytes(sys, order, n_cols);
  if (workspace_bytes < need)
    return fail(SCP_EINVAL, "workspace_bytes " + std::to_string(workspace_bytes) + " below the " +
                                std::to_string(need) + " the product-formula adjoint needs");
  return launch_trotter_adjoint(sys, order, n_cols, workspace, (const double2*)psi0,
                                (const double2*)cotangent, grad_out, (hipStream_t)stream);
}

scp_status scp_propagate_trotter_adjoint_final(scp_system* sys, int32_t order, int32_t n_cols,
                                               void* workspace, size_t workspace_bytes,
                                               const void* psiT, const void* cotangent,
                                               double* grad_out, void* stream) {
  g_err.clear();
  if (!sys || !workspace || !psiT || !cotangent || !grad_out) return fail(SCP_EINVAL, "null argument");
  if (n_cols < 1) return fail(SCP_EINVAL, "n_cols must be >= 1");
  scp_status st = trotter_adjoint_check(sys, order);
  if (st != SCP_OK) return st;
  const size_t need = trotter_adjoint_workspace_bytes(sys, order, n_cols);
  if (workspace_bytes < need)
    return fail(SCP_EINVAL, "workspace_bytes " + std::to_string(workspace_bytes) + " below the " +
                                std::to_string(need) + " the product-formula adjoint needs");
  return launch_trotter_adjoint_final(sys, order, n_cols, workspace, (const double2*)psiT,
                                      (const double2*)cotangent, grad_out, (hipStream_t)stream);
}

scp_status scp_fidelity(const void* U, int64_t D, int32_t S, int32_t precision, int32_t d_c,
                        const int64_t* comp_rows, const int32_t* comp_cols, const void* target,
                        void* tau_out, void* cotangent, double* F_out, void* stream) {
  g_err.clear();
  if (!U || !comp_rows || !comp_cols || !target || !tau_out) return fail(SCP_EINVAL, "null argument");
  if (D < 1 || S < 1 || d_c < 1 || (precision != 0 && precision != 1))
    return fail(SCP_EINVAL, "bad sizes");
  hipStream_t st = (hipStream_t)stream;
  scp_status s = launch_fidelity(U, D, S, precision, d_c, comp_rows, comp_cols, target, tau_out,
                                 cotangent, st);
  if (s != SCP_OK) return s;
  if (F_out) {
    double2 tau;
    HIPCHK(hipMemcpyAsync(&tau, tau_out, sizeof(double2), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *F_out = (tau.x * tau.x + tau.y * tau.y) / ((double)d_c * d_c);
    if (!std::isfinite(*F_out)) return fail(SCP_ENONFINITE, "fidelity is not finite");
  }
  return SCP_OK;
}

scp_status scp_fidelity_states(const void* U, int64_t D, int32_t S, int32_t precision,
                               int32_t n_t, const int32_t* cols, const void* targets,
                               void* tau_out, void* cotangent, double* F_out, void* stream) {
  g_err.clear();
  if (!U || !cols || !targets || !tau_out) return fail(SCP_EINVAL, "null argument");
  if (D < 1 || S < 1 || n_t < 1 || (precision != 0 && precision != 1))
    return fail(SCP_EINVAL, "bad sizes");
  hipStream_t st = (hipStream_t)stream;
  scp_status s = launch_fidelity_states(U, D, S, precision, n_t, cols, targets, tau_out, cotangent,
                                        st);
  if (s != SCP_OK) return s;
  if (F_out) {
    double2 tau;
    HIPCHK(hipMemcpyAsync(&tau, tau_out, sizeof(double2), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *F_out = (tau.x * tau.x + tau.y * tau.y) / ((double)n_t * n_t);
    if (!std::isfinite(*F_out)) return fail(SCP_ENONFINITE, "fidelity is not finite");
  }
  return SCP_OK;
}

scp_status scp_fidelity_local(const void* U, int64_t D, int32_t S, int32_t precision,
                              int32_t n_qubits, const int32_t* cols, const void* W,
                              const int64_t* comp_rows, const void* target, int32_t mode,
                              void* block_out, void* tau_out, double* F_out, double* params_out,
                              void* cotangent, void* stream) {
  g_err.clear();
  if (!U || !cols || !target || !block_out || !F_out || (!W && !comp_rows))
    return fail(SCP_EINVAL, "null argument");
  if (D < 1 || S < 1 || n_qubits < 1 || n_qubits > 6 || (precision != 0 && precision != 1))
    return fail(SCP_EINVAL, "bad sizes (n_qubits must be 1..6)");
  if (mode != 1 && mode != 2) return fail(SCP_EINVAL, "mode must be 1 (Z phases) or 2 (SU(2))");
  return launch_fidelity_local(U, D, S, precision, n_qubits, cols, W, comp_rows, target, mode,
                               block_out, tau_out, F_out, params_out, cotangent,
                               (hipStream_t)stream);
}

scp_status scp_fidelity_zcomp(const void* U, int64_t D, int32_t S, int32_t precision,
                              int32_t n_qubits, const int64_t* comp_rows, const int32_t* comp_cols,
                              const void* target, void* block_out, void* tau_out, double* F_out,
                              double* phases_out, void* cotangent, void* stream) {
  g_err.clear();
  if (!U || !comp_rows || !comp_cols || !target || !block_out || !F_out)
    return fail(SCP_EINVAL, "null argument");
  if (D < 1 || S < 1 || n_qubits < 1 || n_qubits > 6 || (precision != 0 && precision != 1))
    return fail(SCP_EINVAL, "bad sizes (n_qubits must be 1..6)");
  return launch_zcomp(U, D, S, precision, n_qubits, comp_rows, comp_cols, target, block_out,
                      tau_out, F_out, phases_out, cotangent, (hipStream_t)stream);
}

scp_status scp_propagate_adjoint(scp_system* sys, const scp_solve_opts* opts, void* workspace,
                                 const void* psi0, const void* cotangent, double* grad_out,
                                 void* stream) {
  g_err.clear();
  if (!sys || !opts || !workspace || !cotangent || !grad_out) return fail(SCP_EINVAL, "null argument");
  if (opts->precision != 0) return fail(SCP_EINVAL, "the adjoint runs on the FP32 path (precision 0)");
  if (opts->n_cols < 1) return fail(SCP_EINVAL, "n_cols must be >= 1");
  if (opts->ckpt_every < 0) return fail(SCP_EINVAL, "ckpt_every must be >= 0");
  WsLayout w = ws_layout(sys, opts, 1);
  if (opts->workspace_bytes < w.total)
    return fail(SCP_EINVAL, "workspace_bytes " + std::to_string(opts->workspace_bytes) +
                                " below the " + std::to_string(w.total) +
                                " the adjoint needs (scp_workspace_size with_grad = 1)");
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  if (w.gather_grad) {
    if (psi0 != nullptr) {
      ck_claim(sys, workspace);
      ck_clear(sys);
      scp_status s = launch_gather_ckpt_forward(sys, opts->n_cols, w.ce, workspace,
                                                opts->workspace_bytes, (const float2*)psi0,
                                                nullptr, st);
      if (s != SCP_OK) return s;
      ck_record(sys, workspace, opts->n_cols, w.ce);
    } else if (!ck_valid(sys, workspace, opts->n_cols, w.ce)) {
      return fail(SCP_EINVAL,
                  "no checkpoints of this system for this workspace and opts: the last "
                  "scp_propagate must run with with_ckpt = 1 on the same workspace, n_cols and "
                  "ckpt_every (or pass psi0)");
    }
    return launch_gather_adjoint(sys, opts->n_cols, w.ce, workspace, opts->workspace_bytes,
                                 (const float2*)cotangent, grad_out, st);
  }
  if (psi0 != nullptr) {
    ck_claim(sys, workspace);
    ck_clear(sys);
    scp_status s = launch_rk4(sys, (const float2*)psi0, nullptr, (float2*)(ws + w.lo),
                              (float4*)(ws + w.ckpt), w.ce, opts->n_cols, st);
    if (s != SCP_OK) return s;
    ck_record(sys, workspace, opts->n_cols, w.ce);
  } else if (!ck_valid(sys, workspace, opts->n_cols, w.ce)) {
    return fail(SCP_EINVAL,
                "no checkpoints of this system for this workspace and opts: the last "
                "scp_propagate must run with with_ckpt = 1 on the same workspace, n_cols and "
                "ckpt_every (or pass psi0)");
  }
  return finish_adjoint(sys, w, ws, cotangent, grad_out, opts->n_cols, st);
}

}  // extern "C"

namespace scp {

scp_status finish_adjoint(scp_system* sys, const WsLayout& w, char* ws, const void* cotangent,
                          double* grad_out, int S, hipStream_t st) {
  scp_status s = launch_adjoint_impl(sys, ws + w.ckpt, cotangent, ws + w.seg, ws + w.lo, ws + w.lam,
                                     ws + w.lamstate, (double*)(ws + w.part), w.ce, w.nckpt,
                                     S, st);
  if (s != SCP_OK) return s;
  const int nacc = sys->plan.nacc;
  std::vector<double> part((size_t)w.nwg * 4 * nacc);
  HIPCHK(hipMemcpyAsync(part.data(), ws + w.part, part.size() * sizeof(double),
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  bool finite = true;
  for (int i = 0; i < nacc; ++i) {
    double a = 0.0;
    for (int b = 0; b < w.nwg; ++b)
      for (int wv = 0; wv < 4; ++wv) a += part[((size_t)b * 4 + wv) * nacc + i];
    grad_out[i] = 2.0 * a;
    finite &= std::isfinite(grad_out[i]);
  }
  if (!finite) return fail(SCP_ENONFINITE, "gradient is not finite");
  return SCP_OK;
}

}  // namespace scp

extern "C" {

// Allocation-free adjoint: the workspace (checkpoints, segment buffer,
// costate, FP64 partials) is a file-scope device array of fixed size.  Each
// device holds its own copy until the process ends; the host reaches it only
// through the address hipGetSymbolAddress returns for the current device,
// taken once per device on the first call there.
#define SCP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
static __device__ __align__(256) unsigned char scratch[SCP_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_ptr;   // device ordinal -> its copy of scratch

static scp_status scratch_address(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr) return fail(SCP_EHIP, "hipGetSymbolAddress(scratch) gave a null address");
    it = g_scratch_ptr.emplace(dev, p).first;
  }
  *out = it->second;
  return SCP_OK;
}

scp_status scp_propagate_adjoint_noalloc(scp_system* sys, const scp_solve_opts* opts,
                                         const void* psi0, const void* cotangent,
                                         double* grad_out, void* stream) {
  g_err.clear();
  if (!sys || !opts || !psi0 || !cotangent || !grad_out) return fail(SCP_EINVAL, "null argument");
  if (opts->precision != 0) return fail(SCP_EINVAL, "the adjoint runs on the FP32 path (precision 0)");
  if (opts->n_cols < 1) return fail(SCP_EINVAL, "n_cols must be >= 1");
  if (opts->ckpt_every < 0) return fail(SCP_EINVAL, "ckpt_every must be >= 0");
  WsLayout w = ws_layout(sys, opts, 1, false);
  if (w.total > SCP_NOALLOC_SCRATCH_BYTES)
    return fail(SCP_EINVAL, "the adjoint needs " + std::to_string(w.total) +
                                " bytes of workspace; the static scratch holds " +
                                std::to_string(SCP_NOALLOC_SCRATCH_BYTES));
  if (sys->timing) return fail(SCP_EINVAL, "kernel timing creates HIP events; switch it off first");
  void* base = nullptr;
  scp_status s = scratch_address(&base);
  if (s != SCP_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)base;
  s = launch_rk4(sys, (const float2*)psi0, nullptr, (float2*)(ws + w.lo), (float4*)(ws + w.ckpt),
                 w.ce, opts->n_cols, st);
  if (s != SCP_OK) return s;
  return finish_adjoint(sys, w, ws, cotangent, grad_out, opts->n_cols, st);
}

void scp_destroy(scp_system* sys) {
  if (!sys) return;
  ck_clear(sys);
  timing_drop(sys);
  if (sys->d_plan) (void)hipFree(sys->d_plan);
  if (sys->d_ops) (void)hipFree(sys->d_ops);
  if (sys->d_ctab) (void)hipFree(sys->d_ctab);
  if (sys->d_dctab) (void)hipFree(sys->d_dctab);
  if (sys->d_dctab64) (void)hipFree(sys->d_dctab64);
  if (sys->d_ctab64) (void)hipFree(sys->d_ctab64);
  if (sys->d_ph) (void)hipFree(sys->d_ph);
  if (sys->d_rops) (void)hipFree(sys->d_rops);
  if (sys->d_scratch) (void)hipFree(sys->d_scratch);
  delete sys;
}

}  // extern "C"
