// Serving runtime: continuous batching of propagation / gradient requests.
//
// Requests (a device description, its columns, a target, and whether the
// gradient is wanted) queue on the host.  Each call of scp_server_step is one
// tick:
//   1. admit queued requests in arrival order while their device footprint
//      (stage tables + states + checkpoints + adjoint buffers) fits the HBM
//      budget and the active count is below max_active;
//   2. advance every active request by one chunk: forward steps, or adjoint
//      segments once the forward is done, with batched launches per size
//      class (d, NR, MP) in which every workgroup reads its own work
//      descriptor (its request's tables and states, its column block, its
//      step range or segment): one forward launch, or per adjoint segment a
//      recompute launch and a reverse launch;
//   3. reduce the fidelity of requests whose forward completed (and seed the
//      costate of gradient requests), finish gradients, release memory.
// With the engine set to 0 or 2, requests that the gather engine runs (few
// columns of a small device, as for scp_propagate) are batched per (d, modes)
// on it instead: one launch per tick of every such request's step range of
// the forward (its compensated state saved between chunks), and per round one
// launch of the next segment of every such request's reverse walk.
// The per-request state (psi hi/lo, costate, per-wave FP64 accumulators) is
// carried between ticks exactly, so a request's result does not depend on
// what else is in flight or on the chunk boundaries.  Every launch is bounded
// (no device-side waiting).  Size classes go round-robin to four worker
// streams so that their launches overlap; a tick ends by synchronising them.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>

#include "internal.h"

namespace scp {

scp_status launch_rk4_batched(int d, int NR, int MP, bool rf, const FwdItem* items, int nitems, int wg,
                              size_t sh, bool recompute, hipStream_t s);
scp_status launch_adjoint_batched(int d, int NR, int MP, bool rf, const AdjItem* items, int nitems, int wg,
                                  size_t sh, hipStream_t s);
size_t adjoint_lds_bytes(const Plan& P);

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Deep copy of a system description (the caller's arrays may go away).
struct DescCopy {
  scp_system_desc desc{};
  std::vector<scp_mode_desc> modes;
  std::vector<scp_coupling_desc> coup;
  std::vector<scp_drive_desc> drives;
  std::vector<std::vector<double>> pars, raw_eps, raw_ops;
  void copy(const scp_system_desc* d) {
    desc = *d;
    modes.assign(d->modes, d->modes + d->n_modes);
    coup.assign(d->couplings, d->couplings + d->n_couplings);
    drives.assign(d->drives, d->drives + d->n_drives);
    raw_eps.resize(modes.size());
    raw_ops.resize(modes.size());
    for (size_t m = 0; m < modes.size(); ++m) {
      if (modes[m].kind == SCP_MODE_RAW && modes[m].raw_eps && modes[m].raw_ops) {
        const int t = modes[m].trunc;
        raw_eps[m].assign(modes[m].raw_eps, modes[m].raw_eps + t);
        raw_ops[m].assign(modes[m].raw_ops, modes[m].raw_ops + 4 * t * t);
        modes[m].raw_eps = raw_eps[m].data();
        modes[m].raw_ops = raw_ops[m].data();
      }
    }
    pars.resize(drives.size());
    for (size_t k = 0; k < drives.size(); ++k) {
      pars[k].assign(drives[k].par, drives[k].par + drives[k].n_par);
      drives[k].par = pars[k].data();
    }
    desc.modes = modes.data();
    desc.couplings = coup.empty() ? nullptr : coup.data();
    desc.drives = drives.empty() ? nullptr : drives.data();
  }
};

enum { RQ_QUEUED = 0, RQ_RUNNING = 1, RQ_DONE = 2, RQ_FAILED = 3 };

struct Request {
  int64_t id = 0;
  DescCopy dc;
  std::vector<int64_t> columns, rows;
  std::vector<int32_t> cols;
  std::vector<double> target;
  int S = 0, d_c = 0, want_grad = 0;
  int state = RQ_QUEUED;
  int phase = 0;          // 0 forward, 1 adjoint
  int n_done = 0, seg_next = 0, ce = 1, nckpt = 1, nwg = 1;
  size_t bytes = 0;
  scp_system* sys = nullptr;
  void* dmem = nullptr;
  float2 *psi = nullptr, *state_hi = nullptr, *lo = nullptr, *segbuf = nullptr, *sum = nullptr,
         *lamstate = nullptr, *cot = nullptr;
  float4* ckpt = nullptr;
  double* part = nullptr;
  int64_t* d_rows = nullptr;
  int32_t* d_cols = nullptr;
  double2* d_target = nullptr;
  double2* d_tau = nullptr;
  double F = 0.0;
  std::vector<double> grad;
  double t_submit = 0, t_admit = 0, t_done = 0;
  std::string err;
  double cost_step = 1.0;   // relative device time of one forward step of one workgroup
  hipStream_t tick_stream = nullptr;   // worker stream of this tick's launch
  bool gather = false;      // runs on the gather engine
  void* gws = nullptr;      // its workspace (inside dmem)
  size_t gws_bytes = 0;
  GServeInfo gi{};          // its device descriptions, state buffer and LDS needs
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace
}  // namespace scp

struct scp_server {
  size_t budget = 0, used = 0;
  int max_active = 64;
  // engine of admissions, as scp_system_set_engine (0 automatic, 1 register,
  // 2 gather); the register-layout kernels by default: batched, they give the
  // higher throughput under load
  int engine = 1;
  double chunk_work = 2.0e7;   // per-tick work budget per workgroup (cost units)
  hipStream_t stream = nullptr;        // admission (builds and uploads)
  static constexpr int kWork = 4;      // one per hardware queue
  hipStream_t work[kWork] = {};        // size classes run concurrently on these
  int64_t next_id = 1;
  std::deque<scp::Request*> queue;
  std::vector<scp::Request*> active;
  std::map<int64_t, std::unique_ptr<scp::Request>> all;
  double t0 = 0;
  // batched work descriptors (device + pinned host staging)
  void* d_items = nullptr;
  void* h_items = nullptr;
  size_t items_cap = 0;
};

namespace scp {
namespace {

// Upper bound of a request's device footprint before its plan exists.
size_t estimate_bytes(const scp_system_desc* d, int S, int want_grad) {
  int dd = 0;   // the system runs at the largest truncation
  for (int m = 0; m < d->n_modes; ++m) dd = std::max(dd, (int)d->modes[m].trunc);
  size_t D = 1;
  for (int m = 0; m < d->n_modes; ++m) D *= (size_t)dd;
  const size_t nslots = 2 * (size_t)d->n_couplings + d->n_drives + 1;
  const size_t npairs = (size_t)d->n_couplings + 1;
  const size_t block_q = (4 * nslots + npairs) * dd * dd;
  size_t npulse = 0;
  for (int k = 0; k < d->n_drives; ++k) npulse += (size_t)d->drives[k].n_par;
  const size_t N = (size_t)d->n_steps;
  size_t b = (2 * N + 1) * block_q * 8 + 3 * N * (d->n_drives + npulse) * 12 + sizeof(Plan);
  const size_t ce = (size_t)std::ceil(std::sqrt((double)N));
  const size_t nck = (N + ce - 1) / ce;
  b += 4 * (size_t)S * D * 8;                               // psi, state_hi, lo, cotangent
  if (want_grad) {
    b += nck * S * D * 16 + ce * 4 * S * D * 8 + 2 * S * D * 8;
    b += (size_t)S * 4 * (npulse + 3 * d->n_modes + d->n_couplings) * 8;
  }
  return b + (1 << 20);
}

scp_status admit(scp_server* sv, Request* r) {
  scp_system* sys = nullptr;
  scp_status st = scp_build_system(&r->dc.desc, sv->stream, &sys);
  if (st != SCP_OK) return st;
  r->sys = sys;
  const Plan& P = sys->plan;
  const size_t S = (size_t)r->S, D = (size_t)sys->D;
  r->ce = (int)std::ceil(std::sqrt((double)sys->n_steps));
  r->nckpt = (sys->n_steps + r->ce - 1) / r->ce;
  r->nwg = (r->S + P.CPW - 1) / P.CPW;
  // the gather engine where scp_propagate would take it and its tables fit
  // the budget beside what is admitted
  r->gather = false;
  if (sv->engine != 1 && (sv->engine == 2 ? gather_supported(sys) : gather_preferred(sys, r->S))) {
    if (gather_grad_check(sys) == SCP_OK) {
      r->gws_bytes = gather_serve_bytes(sys, r->S, r->ce, r->want_grad != 0);
      r->gather = r->gws_bytes > 0 &&
                  sv->used + r->gws_bytes + (size_t)(4 << 20) + 2 * (size_t)r->S * sys->D * 8 <=
                      sv->budget;
    } else {
      set_error("");
    }
  }
  size_t off = 0;
  auto take = [&](size_t n) {
    size_t o = off;
    off = align256(off + n);
    return o;
  };
  const size_t o_psi = take(S * D * 8), o_hi = take(S * D * 8), o_lo = take(S * D * 8),
               o_cot = take(S * D * 8), o_rows = take(r->d_c * 8), o_cols = take(r->d_c * 4),
               o_tgt = take((size_t)r->d_c * r->d_c * 16), o_tau = take(16);
  size_t o_ck = 0, o_seg = 0, o_sum = 0, o_ls = 0, o_part = 0, o_g = 0;
  if (r->gather) {
    o_g = take(r->gws_bytes);
  } else if (r->want_grad) {
    o_ck = take((size_t)r->nckpt * S * D * 16);
    o_seg = take((size_t)r->ce * 4 * S * D * 8);
    o_sum = take(S * D * 8);
    o_ls = take(S * D * 8);
    o_part = take((size_t)r->nwg * 4 * std::max(1, P.nacc) * 8);
  }
  if (hipMalloc(&r->dmem, off) != hipSuccess) {
    scp_destroy(sys);
    r->sys = nullptr;
    return fail(SCP_ENOMEM, "request allocation");
  }
  r->bytes = off;
  char* b = (char*)r->dmem;
  r->psi = (float2*)(b + o_psi);
  r->state_hi = (float2*)(b + o_hi);
  r->lo = (float2*)(b + o_lo);
  r->cot = (float2*)(b + o_cot);
  r->d_rows = (int64_t*)(b + o_rows);
  r->d_cols = (int32_t*)(b + o_cols);
  r->d_target = (double2*)(b + o_tgt);
  r->d_tau = (double2*)(b + o_tau);
  if (r->gather) r->gws = b + o_g;
  if (!r->gather && r->want_grad) {
    r->ckpt = (float4*)(b + o_ck);
    r->segbuf = (float2*)(b + o_seg);
    r->sum = (float2*)(b + o_sum);
    r->lamstate = (float2*)(b + o_ls);
    r->part = (double*)(b + o_part);
  }
  // initial states: basis columns
  std::vector<float2> h(S * D, make_float2(0.f, 0.f));
  for (size_t j = 0; j < S; ++j) h[j * D + (size_t)r->columns[j]] = make_float2(1.f, 0.f);
  hipMemcpyAsync(r->psi, h.data(), h.size() * 8, hipMemcpyHostToDevice, sv->stream);
  hipMemcpyAsync(r->d_rows, r->rows.data(), r->rows.size() * 8, hipMemcpyHostToDevice, sv->stream);
  hipMemcpyAsync(r->d_cols, r->cols.data(), r->cols.size() * 4, hipMemcpyHostToDevice, sv->stream);
  hipMemcpyAsync(r->d_target, r->target.data(), r->target.size() * 8, hipMemcpyHostToDevice,
                 sv->stream);
  if (r->gather) {
    scp_status gs = gather_serve_prepare(sys, r->S, r->ce, r->want_grad != 0, r->gws, r->gws_bytes,
                                         r->psi, r->psi, r->cot, sv->stream);
    if (gs == SCP_OK) gs = gather_serve_info(sys, r->S, r->ce, r->want_grad != 0, r->gws, r->gi);
    if (gs != SCP_OK) return gs;
  }
  if (hipStreamSynchronize(sv->stream) != hipSuccess) return fail(SCP_EHIP, "admission copy");
  r->cost_step = (double)P.CPW * P.D * (P.L * 2.0 + 4.0 * P.MP);
  r->state = RQ_RUNNING;
  r->phase = 0;
  r->n_done = 0;
  r->t_admit = now_s() - sv->t0;
  return SCP_OK;
}

void release(scp_server* sv, Request* r) {
  if (r->dmem) (void)hipFree(r->dmem);
  r->dmem = nullptr;
  if (r->sys) scp_destroy(r->sys);
  r->sys = nullptr;
  sv->used -= std::min(sv->used, r->bytes);
}

scp_status ensure_items(scp_server* sv, size_t bytes) {
  if (bytes <= sv->items_cap) return SCP_OK;
  if (sv->d_items) (void)hipFree(sv->d_items);
  if (sv->h_items) (void)hipHostFree(sv->h_items);
  sv->d_items = sv->h_items = nullptr;
  sv->items_cap = 0;
  const size_t cap = std::max(bytes, (size_t)1 << 20);
  if (hipMalloc(&sv->d_items, cap) != hipSuccess) return fail(SCP_ENOMEM, "item buffer");
  if (hipHostMalloc(&sv->h_items, cap) != hipSuccess) return fail(SCP_ENOMEM, "item staging");
  sv->items_cap = cap;
  return SCP_OK;
}

}  // namespace
}  // namespace scp

using namespace scp;

extern "C" {

scp_status scp_server_create(size_t hbm_budget_bytes, int32_t max_active, double chunk_work,
                             void* stream, scp_server** out) {
  if (!out || hbm_budget_bytes == 0 || max_active < 1) return fail(SCP_EINVAL, "bad server options");
  scp_server* sv = new (std::nothrow) scp_server();
  if (!sv) return fail(SCP_ENOMEM, "host allocation");
  sv->budget = hbm_budget_bytes;
  sv->max_active = max_active;
  if (chunk_work > 0) sv->chunk_work = chunk_work;
  sv->stream = (hipStream_t)stream;
  for (int i = 0; i < scp_server::kWork; ++i)
    if (hipStreamCreateWithFlags(&sv->work[i], hipStreamNonBlocking) != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipStreamDestroy(sv->work[j]);
      delete sv;
      return fail(SCP_EHIP, "worker stream creation");
    }
  sv->t0 = now_s();
  *out = sv;
  return SCP_OK;
}

scp_status scp_request_bytes(const scp_system_desc* desc, int32_t n_cols, int32_t want_grad,
                             size_t* bytes) {
  if (!desc || !bytes || n_cols < 1 || desc->n_modes < 1 || !desc->modes)
    return fail(SCP_EINVAL, "null or empty argument");
  *bytes = estimate_bytes(desc, n_cols, want_grad ? 1 : 0);
  return SCP_OK;
}

scp_status scp_server_submit(scp_server* sv, const scp_system_desc* desc, const int64_t* columns,
                             int32_t n_cols, const int64_t* comp_rows, const int32_t* comp_cols,
                             int32_t d_c, const double* target, int32_t want_grad,
                             int64_t* id_out) {
  if (!sv || !desc || !columns || n_cols < 1 || !comp_rows || !comp_cols || d_c < 1 || !target ||
      !id_out)
    return fail(SCP_EINVAL, "null or empty argument");
  auto r = std::make_unique<Request>();
  r->dc.copy(desc);
  int dmax = 0;   // the system runs at the largest truncation (see scp_mode_desc)
  for (int m = 0; m < desc->n_modes; ++m) dmax = std::max(dmax, (int)desc->modes[m].trunc);
  int64_t D = 1;
  for (int m = 0; m < desc->n_modes; ++m) D *= dmax;
  for (int j = 0; j < n_cols; ++j)
    if (columns[j] < 0 || columns[j] >= D) return fail(SCP_EINVAL, "column index out of range");
  for (int i = 0; i < d_c; ++i) {
    if (comp_rows[i] < 0 || comp_rows[i] >= D) return fail(SCP_EINVAL, "comp row out of range");
    if (comp_cols[i] < 0 || comp_cols[i] >= n_cols) return fail(SCP_EINVAL, "comp col out of range");
  }
  r->columns.assign(columns, columns + n_cols);
  r->rows.assign(comp_rows, comp_rows + d_c);
  r->cols.assign(comp_cols, comp_cols + d_c);
  r->target.assign(target, target + 2 * (size_t)d_c * d_c);
  r->S = n_cols;
  r->d_c = d_c;
  r->want_grad = want_grad ? 1 : 0;
  r->bytes = estimate_bytes(desc, n_cols, r->want_grad);
  if (r->bytes > sv->budget) return fail(SCP_EBUSY, "request larger than the HBM budget");
  r->id = sv->next_id++;
  r->t_submit = now_s() - sv->t0;
  *id_out = r->id;
  sv->queue.push_back(r.get());
  sv->all[r->id] = std::move(r);
  return SCP_OK;
}

scp_status scp_server_step(scp_server* sv, int32_t* n_active, int32_t* n_queued) {
  if (!sv) return fail(SCP_EINVAL, "null server");
  // 1. admission by footprint, in arrival order
  while (!sv->queue.empty() && (int)sv->active.size() < sv->max_active) {
    Request* r = sv->queue.front();
    const size_t est = r->bytes;
    if (sv->used + est > sv->budget) break;
    sv->queue.pop_front();
    scp_status s = admit(sv, r);
    if (s != SCP_OK) {
      r->state = RQ_FAILED;
      r->err = scp_last_error();
      release(sv, r);
      continue;
    }
    sv->used += std::max(est, r->bytes);
    r->bytes = std::max(est, r->bytes);
    sv->active.push_back(r);
  }
  if (!sv->active.empty()) {
    // 2. one chunk for everyone, one launch per (kind, size class)
    struct Work { Request* r; int n0, n1, s_hi, s_lo; };
    // (kind, d, NR, MP, real frame)
    std::map<std::tuple<int, int, int, int, int>, std::vector<Work>> classes;
    for (Request* r : sv->active) {
      if (r->gather) continue;
      const Plan& P = r->sys->plan;
      const double per_wg_step = r->cost_step;
      const int steps = std::max(8, (int)(sv->chunk_work / per_wg_step));
      if (r->phase == 0) {
        const int n0 = r->n_done, n1 = std::min(r->sys->n_steps, n0 + steps);
        classes[{0, P.d, P.NR, P.MP, P.real_frame}].push_back({r, n0, n1, 0, 0});
      } else {
        const int segs = std::max(1, steps / (4 * r->ce));
        const int s_hi = r->seg_next, s_lo = std::max(0, s_hi - segs + 1);
        classes[{1, P.d, P.NR, P.MP, P.real_frame}].push_back({r, 0, 0, s_hi, s_lo});
      }
    }
    // staging: per class, the forward items, or per adjoint round (one segment
    // of every request that has one left this tick) recompute + reverse items
    size_t need = 0;
    for (auto& kv : classes) {
      size_t rounds = 1;
      for (auto& w : kv.second) {
        const size_t rw = std::get<0>(kv.first) == 0 ? 1 : (size_t)(w.s_hi - w.s_lo + 1);
        need += rw * w.r->nwg * (sizeof(FwdItem) + sizeof(AdjItem));
        rounds = std::max(rounds, rw);
      }
      need += 2 * 256 * rounds;   // alignment of every upload
    }
    // the gather-engine requests' items (batched below)
    for (Request* r : sv->active)
      if (r->gather) {
        const int steps = std::max(8, (int)(sv->chunk_work / r->cost_step));
        const size_t rounds = r->phase == 0 ? 1 : (size_t)std::max(1, steps / r->ce);
        need += rounds * (2 * (size_t)r->S * sizeof(GItem) + 2 * 256);
      }
    scp_status s = ensure_items(sv, need);
    if (s != SCP_OK) return s;
    size_t off = 0;
    int ci = 0;
    // upload n items at off and return the device pointer
    auto stage = [&](const void* host, size_t bytes, hipStream_t st, void** dptr) -> bool {
      *dptr = (char*)sv->d_items + off;
      if (hipMemcpyAsync(*dptr, host, bytes, hipMemcpyHostToDevice, st) != hipSuccess) return false;
      off += align256(bytes);
      return true;
    };
    for (auto& kv : classes) {
      hipStream_t st = sv->work[ci++ % scp_server::kWork];
      const int kind = std::get<0>(kv.first), d = std::get<1>(kv.first), NR = std::get<2>(kv.first),
                MP = std::get<3>(kv.first);
      const bool rf = std::get<4>(kv.first) != 0;
      int wg = 64;
      size_t sh_f = 0, sh_a = 0;
      for (auto& w : kv.second) {
        const Plan& P = w.r->sys->plan;
        wg = std::max(wg, P.WG);
        sh_f = std::max(sh_f, sizeof(float2) * 3 * (size_t)P.CPW * P.D);
        sh_a = std::max(sh_a, adjoint_lds_bytes(P));
      }
      if (kind == 0) {
        FwdItem* it = (FwdItem*)((char*)sv->h_items + off);
        int nit = 0;
        for (auto& w : kv.second) {
          Request* r = w.r;
          for (int cb = 0; cb < r->nwg; ++cb)
            it[nit++] = FwdItem{r->sys->d_plan, r->sys->d_ops, r->sys->d_ctab,
                                w.n0 == 0 ? r->psi : nullptr,
                                w.n1 == r->sys->n_steps ? r->psi : nullptr, r->state_hi, r->lo,
                                r->want_grad ? r->ckpt : nullptr, nullptr, nullptr,
                                r->sys->d_ph, r->sys->d_rops, r->ce, r->S, cb, w.n0, w.n1, 0};
        }
        void* dptr = nullptr;
        if (!stage(it, (size_t)nit * sizeof(FwdItem), st, &dptr)) return fail(SCP_EHIP, "item upload");
        s = launch_rk4_batched(d, NR, MP, rf, (const FwdItem*)dptr, nit, wg, sh_f, false, st);
        if (s != SCP_OK) return s;
      } else {
        // round j: segment s_hi - j of every request that still has one this tick
        int rounds = 0;
        for (auto& w : kv.second) rounds = std::max(rounds, w.s_hi - w.s_lo + 1);
        for (int j = 0; j < rounds; ++j) {
          FwdItem* fi = (FwdItem*)((char*)sv->h_items + off);
          int nf = 0;
          for (auto& w : kv.second) {
            Request* r = w.r;
            const int seg = w.s_hi - j;
            if (seg < w.s_lo) continue;
            const int n0 = seg * r->ce, n1 = std::min(n0 + r->ce, r->sys->n_steps);
            for (int cb = 0; cb < r->nwg; ++cb)
              fi[nf++] = FwdItem{r->sys->d_plan, r->sys->d_ops, r->sys->d_ctab, nullptr, nullptr,
                                 nullptr, r->lo, nullptr,
                                 r->ckpt + (size_t)seg * r->S * r->sys->D, r->segbuf,
                                 r->sys->d_ph, r->sys->d_rops, 1, r->S, cb, n0, n1, 0};
          }
          void* dptr = nullptr;
          if (!stage(fi, (size_t)nf * sizeof(FwdItem), st, &dptr)) return fail(SCP_EHIP, "item upload");
          s = launch_rk4_batched(d, NR, MP, rf, (const FwdItem*)dptr, nf, wg, sh_f, true, st);
          if (s != SCP_OK) return s;
          AdjItem* ai = (AdjItem*)((char*)sv->h_items + off);
          int na = 0;
          for (auto& w : kv.second) {
            Request* r = w.r;
            const int seg = w.s_hi - j;
            if (seg < w.s_lo) continue;
            for (int cb = 0; cb < r->nwg; ++cb)
              ai[na++] = AdjItem{r->sys->d_plan, r->sys->d_ops, r->sys->d_ctab, r->sys->d_dctab,
                                 r->ckpt, r->cot, r->segbuf, r->lo, r->sum, r->lamstate, r->part,
                                 r->sys->d_ph, r->sys->d_rops, r->ce, r->nckpt, r->S, cb, seg, seg,
                                 seg == r->nckpt - 1 ? 1 : 0, 0};
          }
          if (!stage(ai, (size_t)na * sizeof(AdjItem), st, &dptr)) return fail(SCP_EHIP, "item upload");
          s = launch_adjoint_batched(d, NR, MP, rf, (const AdjItem*)dptr, na, wg, sh_a, st);
          if (s != SCP_OK) return s;
        }
      }
      for (auto& w : kv.second) {
        if (kind == 0) w.r->n_done = w.n1;
        else w.r->seg_next = w.s_lo - 1;
        w.r->tick_stream = st;
      }
    }
    // gather-engine requests, batched per (kind, d, modes, checkpoints)
    {
      std::map<std::tuple<int, int, int, int>, std::vector<Request*>> gcls;
      for (Request* r : sv->active)
        if (r->gather)
          gcls[{r->phase, r->sys->d, r->sys->n_modes, r->want_grad}].push_back(r);
      for (auto& kv : gcls) {
        hipStream_t st = sv->work[ci++ % scp_server::kWork];
        const int kind = std::get<0>(kv.first), d = std::get<1>(kv.first),
                  N = std::get<2>(kv.first);
        const bool ck = std::get<3>(kv.first) != 0;
        if (kind == 0) {
          GItem* it = (GItem*)((char*)sv->h_items + off);
          int nit = 0;
          size_t lds = 0;
          for (Request* r : kv.second) {
            const int steps = std::max(8, (int)(sv->chunk_work / r->cost_step));
            const int n0 = r->n_done, n1 = std::min(r->sys->n_steps, n0 + steps);
            for (int c = 0; c < r->S; ++c)
              it[nit++] = GItem{r->gi.A, ck ? r->gi.B : nullptr, n0 == 0 ? nullptr : r->gi.state,
                                r->gi.state, c, n0, n1, 0};
            lds = std::max(lds, r->gi.lds_fwd);
            r->n_done = n1;
            r->tick_stream = st;
          }
          void* dptr = nullptr;
          if (!stage(it, (size_t)nit * sizeof(GItem), st, &dptr)) return fail(SCP_EHIP, "item upload");
          s = gather_launch_fwd_batched(d, N, ck, (const GItem*)dptr, nit, lds, st);
          if (s != SCP_OK) return s;
        } else {
          // round j: launch seg_next - j of every request that still has one this tick
          int rounds = 0;
          std::vector<int> g_lo(kv.second.size());
          for (size_t q = 0; q < kv.second.size(); ++q) {
            Request* r = kv.second[q];
            const int steps = std::max(8, (int)(sv->chunk_work / r->cost_step));
            const int launches = std::max(1, steps / r->ce);
            g_lo[q] = std::max(0, r->seg_next - launches + 1);
            rounds = std::max(rounds, r->seg_next - g_lo[q] + 1);
          }
          for (int j = 0; j < rounds; ++j) {
            GItem* it = (GItem*)((char*)sv->h_items + off);
            int nit = 0;
            size_t lds = 0;
            for (size_t q = 0; q < kv.second.size(); ++q) {
              Request* r = kv.second[q];
              const int gs = r->seg_next - j;
              if (gs < g_lo[q]) continue;
              for (int b = 0; b < 2 * r->S; ++b)
                it[nit++] = GItem{r->gi.A, r->gi.B, nullptr, nullptr, b, 0, 0, gs};
              lds = std::max(lds, r->gi.lds_adj);
            }
            void* dptr = nullptr;
            if (!stage(it, (size_t)nit * sizeof(GItem), st, &dptr))
              return fail(SCP_EHIP, "item upload");
            s = gather_launch_adj_batched(d, N, (const GItem*)dptr, nit, lds, st);
            if (s != SCP_OK) return s;
          }
          for (size_t q = 0; q < kv.second.size(); ++q) {
            kv.second[q]->seg_next = g_lo[q] - 1;
            kv.second[q]->tick_stream = st;
          }
        }
      }
    }
    // 3. fidelity (and costate) for forward completions
    for (Request* r : sv->active)
      if (r->phase == 0 && r->n_done == r->sys->n_steps) {
        s = launch_fidelity(r->psi, r->sys->D, r->S, 0, r->d_c, r->d_rows, r->d_cols, r->d_target,
                            r->d_tau, r->want_grad ? (void*)r->cot : nullptr, r->tick_stream);
        if (s != SCP_OK) return s;
      }
    for (int i = 0; i < scp_server::kWork; ++i)
      if (hipStreamSynchronize(sv->work[i]) != hipSuccess)
        return fail(SCP_EHIP, "tick synchronisation");
    const double t = now_s() - sv->t0;
    std::vector<Request*> keep;
    for (Request* r : sv->active) {
      bool done = false;
      if (r->phase == 0 && r->n_done == r->sys->n_steps) {
        double2 tau;
        (void)hipMemcpy(&tau, r->d_tau, sizeof(tau), hipMemcpyDeviceToHost);
        r->F = (tau.x * tau.x + tau.y * tau.y) / ((double)r->d_c * r->d_c);
        if (r->want_grad) {
          r->phase = 1;
          // the gather engine's reverse launches run nckpt down to 0 (the
          // first recomputes the last segment only)
          r->seg_next = r->gather ? gather_serve_nckpt(r->sys, r->ce) : r->nckpt - 1;
        } else {
          done = true;
        }
      } else if (r->phase == 1 && r->seg_next < 0 && r->gather) {
        s = gather_serve_gradient(r->sys, r->S, r->ce, r->gws, r->grad, sv->stream);
        if (s != SCP_OK) return s;
        done = true;
      } else if (r->phase == 1 && r->seg_next < 0) {
        const int nacc = r->sys->plan.nacc;
        std::vector<double> part((size_t)r->nwg * 4 * nacc);
        (void)hipMemcpy(part.data(), r->part, part.size() * 8, hipMemcpyDeviceToHost);
        r->grad.assign(nacc, 0.0);
        for (int i = 0; i < nacc; ++i) {
          double a = 0.0;
          for (int b = 0; b < r->nwg; ++b)
            for (int wv = 0; wv < 4; ++wv) a += part[((size_t)b * 4 + wv) * nacc + i];
          r->grad[i] = 2.0 * a;
        }
        done = true;
      }
      if (done) {
        r->state = (std::isfinite(r->F) ? RQ_DONE : RQ_FAILED);
        r->t_done = t;
        release(sv, r);
      } else {
        keep.push_back(r);
      }
    }
    sv->active.swap(keep);
  }
  if (n_active) *n_active = (int32_t)sv->active.size();
  if (n_queued) *n_queued = (int32_t)sv->queue.size();
  return SCP_OK;
}

scp_status scp_server_result(scp_server* sv, int64_t id, int32_t* state, double* F, double* grad,
                             int32_t* n_params, double* t_submit, double* t_admit,
                             double* t_done) {
  if (!sv) return fail(SCP_EINVAL, "null server");
  auto it = sv->all.find(id);
  if (it == sv->all.end()) return fail(SCP_EINVAL, "unknown request id");
  Request* r = it->second.get();
  if (state) *state = r->state;
  if (F) *F = r->F;
  if (n_params) *n_params = (int32_t)r->grad.size();
  if (grad && r->state == RQ_DONE)
    std::copy(r->grad.begin(), r->grad.end(), grad);
  if (t_submit) *t_submit = r->t_submit;
  if (t_admit) *t_admit = r->t_admit;
  if (t_done) *t_done = r->t_done;
  if (r->state == RQ_FAILED) return fail(SCP_EINVAL, "request failed: " + r->err);
  return SCP_OK;
}

scp_status scp_server_set_engine(scp_server* sv, int32_t engine) {
  if (!sv || engine < 0 || engine > 2) return fail(SCP_EINVAL, "engine must be 0, 1 or 2");
  sv->engine = engine;
  return SCP_OK;
}

void scp_server_destroy(scp_server* sv) {
  if (!sv) return;
  for (Request* r : sv->active) release(sv, r);
  if (sv->d_items) (void)hipFree(sv->d_items);
  if (sv->h_items) (void)hipHostFree(sv->h_items);
  for (int i = 0; i < scp_server::kWork; ++i)
    if (sv->work[i]) (void)hipStreamDestroy(sv->work[i]);
  delete sv;
}

}  // extern "C"
