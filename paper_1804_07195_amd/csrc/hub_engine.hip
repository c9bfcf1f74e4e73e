// Host orchestration of the solves: workspace pool, the batched engine that runs
// FP64 CG (Sec. 3) and the flexible GMRES with single-precision CG preconditioning
// of Appendix A (Algorithm A.1) for many systems at once, and the small Hessenberg
// least-squares problem of the FGMRES update.
#include <algorithm>
#include <map>
#include <cmath>
#include <cstring>

#include "hub_engine.h"

namespace hub {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string t_err;
void set_error(const std::string& msg) { t_err = msg; }
const char* get_error() { return t_err.c_str(); }

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
Geom make_geom(const hub_lattice& lat) {
  Geom g{};
  g.L1 = lat.L1;
  g.L2 = lat.L2;
  g.Nt = lat.Nt;
  g.P = lat.L1 * lat.L2;
  g.n = 2 * g.P * lat.Nt;
  g.dL2 = make_fastdiv((uint32_t)lat.L2);
  g.dL1 = make_fastdiv((uint32_t)lat.L1);
  g.kappa = lat.kappa_t;
  g.ms = lat.ms_t;
  return g;
}

int ntiles_of(int n) { return (n + kTile - 1) / kTile; }

// ---------------------------------------------------------------------------
// Pool
// ---------------------------------------------------------------------------
static constexpr size_t kGran = size_t(2) << 20;

size_t Pool::rounded(size_t bytes) {
  if (bytes >= kGran) return (bytes + kGran - 1) / kGran * kGran;
  size_t r = 4096;
  while (r < bytes) r <<= 1;
  return r;
}

Pool::Pool(int device, size_t budget) : device_(device), budget_(budget) {}

Pool::~Pool() {
  (void)hipSetDevice(device_);
  for (auto& b : free_) {
    drop_event(b.ev, true);
    (void)hipFree(b.p);
  }
  for (auto& l : live_) (void)hipFree(l.first);
}

void Pool::drop_event(SharedEvent* e, bool wait) {
  if (!e) return;
  if (wait && e->ev) (void)hipEventSynchronize(e->ev);
  if (--e->refs == 0) {
    if (e->ev) (void)hipEventDestroy(e->ev);
    delete e;
  }
}

size_t Pool::in_use() const {
  std::lock_guard<std::mutex> lk(mu_);
  return used_;
}

size_t Pool::reserved() const {
  std::lock_guard<std::mutex> lk(mu_);
  return reserved_;
}

void* Pool::alloc(size_t bytes, hipStream_t st) {
  const size_t sz = rounded(bytes == 0 ? 1 : bytes);
  std::lock_guard<std::mutex> lk(mu_);
  // reuse a cached block of the same size: at once on the stream that released it,
  // on another stream once the work before the release has finished
  for (size_t k = 0; k < free_.size(); ++k) {
    Block& b = free_[k];
    if (b.bytes != sz) continue;
    if (b.st != st && b.ev && b.ev->ev && hipEventQuery(b.ev->ev) != hipSuccess) continue;
    void* p = b.p;
    drop_event(b.ev, false);
    free_.erase(free_.begin() + (long)k);
    live_.emplace_back(p, sz);
    used_ += sz;
    return p;
  }
  // release cached blocks until the new one fits
  while (reserved_ + sz > budget_ && !free_.empty()) {
    Block b = free_.back();
    free_.pop_back();
    drop_event(b.ev, true);
    (void)hipFree(b.p);
    reserved_ -= b.bytes;
  }
  if (reserved_ + sz > budget_) {
    set_error("workspace of " + std::to_string(sz) + " bytes exceeds the HBM budget (" +
              std::to_string(reserved_) + " of " + std::to_string(budget_) + " bytes reserved)");
    return nullptr;
  }
  void* p = nullptr;
  if (hipMalloc(&p, sz) != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc of " + std::to_string(sz) + " bytes failed");
    return nullptr;
  }
  reserved_ += sz;
  used_ += sz;
  live_.emplace_back(p, sz);
  return p;
}

void Pool::release(void* p, hipStream_t st) {
  if (p) release_all(std::vector<void*>{p}, st);
}

void Pool::release_all(const std::vector<void*>& ps, hipStream_t st) {
  std::lock_guard<std::mutex> lk(mu_);
  SharedEvent* e = nullptr;
  for (void* p : ps) {
    if (!p) continue;
    for (size_t k = 0; k < live_.size(); ++k) {
      if (live_[k].first != p) continue;
      if (!e) {
        e = new SharedEvent;
        if (hipEventCreateWithFlags(&e->ev, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(e->ev, st) != hipSuccess) {
          // no event to order later users after the stream's work: wait for it here
          if (e->ev) (void)hipEventDestroy(e->ev);
          e->ev = nullptr;
          (void)hipStreamSynchronize(st);
        }
      }
      e->refs++;
      free_.push_back(Block{p, live_[k].second, st, e});
      used_ -= live_[k].second;
      live_.erase(live_.begin() + (long)k);
      break;
    }
  }
}

// ---------------------------------------------------------------------------
// least squares  min | beta e_1 - H y |  for a (k+1) x k upper Hessenberg H
// (Algorithm A.1 solves the normal equations by Cholesky; Givens rotations give
// the same minimiser with better conditioning).
// ---------------------------------------------------------------------------
std::vector<std::complex<double>> hessenberg_lsq(const std::vector<std::complex<double>>& Hin, int ldh, int k,
                                                 double beta, double* resid) {
  using cd = std::complex<double>;
  std::vector<cd> H(Hin);
  std::vector<cd> gvec(k + 1, cd(0.0));
  gvec[0] = beta;
  auto at = [&](int i, int j) -> cd& { return H[(size_t)j * ldh + i]; };
  for (int i = 0; i < k; ++i) {
    const cd a = at(i, i), b = at(i + 1, i);
    const double r = std::sqrt(std::norm(a) + std::norm(b));
    if (r == 0.0) continue;
    double c;
    cd s;
    if (std::abs(a) == 0.0) {
      c = 0.0;
      s = 1.0;
    } else {
      c = std::abs(a) / r;
      s = (a / std::abs(a)) * std::conj(b) / r;
    }
    for (int j = i; j < k; ++j) {
      const cd u = at(i, j), v = at(i + 1, j);
      at(i, j) = c * u + s * v;
      at(i + 1, j) = -std::conj(s) * u + c * v;
    }
    const cd u = gvec[i], v = gvec[i + 1];
    gvec[i] = c * u + s * v;
    gvec[i + 1] = -std::conj(s) * u + c * v;
  }
  // the rotated right-hand side's last entry is the minimal residual
  if (resid) *resid = std::abs(gvec[k]);
  std::vector<cd> y(k, cd(0.0));
  for (int i = k - 1; i >= 0; --i) {
    cd acc = gvec[i];
    for (int j = i + 1; j < k; ++j) acc -= at(i, j) * y[j];
    y[i] = at(i, i) == cd(0.0) ? cd(0.0) : acc / at(i, i);
  }
  return y;
}

// ---------------------------------------------------------------------------
// Engine
// ---------------------------------------------------------------------------
enum Phase : int {
  PH_NEW = 0,
  PH_CG_ITER,
  PH_CG_CONFIRM,
  PH_F_INNER,
  PH_F_POST_INIT,
  PH_F_ARNOLDI,
  PH_F_POST_ARNOLDI,
  PH_F_LSQ,
  PH_DONE
};

#define HUB_TRY(expr)                        \
  do {                                       \
    hipError_t e_ = (expr);                  \
    if (e_ != hipSuccess) return e_;         \
  } while (0)

Engine::Engine(Pool* pool, hipStream_t st) : pool_(pool), st_(st), slots_(kMaxSys, nullptr) {
  ok_ = hipMalloc(&d_desc_, sizeof(SysDesc) * kMaxSys) == hipSuccess &&
        hipHostMalloc(&h_desc_, sizeof(SysDesc) * kMaxSys, hipHostMallocDefault) == hipSuccess &&
        hipMalloc(&d_y_, sizeof(double) * kYStride * kMaxSys) == hipSuccess &&
        hipHostMalloc(&h_y_, sizeof(double) * kYStride * kMaxSys, hipHostMallocDefault) == hipSuccess &&
        hipMalloc(&d_scal_, sizeof(Scal) * kMaxSys) == hipSuccess &&
        hipHostMalloc(&h_scal_, sizeof(Scal) * kMaxSys, hipHostMallocDefault) == hipSuccess &&
        hipHostMalloc(&h_flags_, sizeof(Scal) * kMaxSys * 4 + 256, hipHostMallocCoherent) == hipSuccess &&
        hipHostMalloc(&h_pub_, sizeof(Scal) * kMaxSys + 256, hipHostMallocCoherent) == hipSuccess &&
        hipMemsetAsync(d_scal_, 0, sizeof(Scal) * kMaxSys, st_) == hipSuccess;
  if (ok_) {
    std::memset(h_scal_, 0, sizeof(Scal) * kMaxSys);
    std::memset(h_pub_, 0, sizeof(Scal) * kMaxSys + 256);
    h_pub_flag_ = reinterpret_cast<unsigned*>(reinterpret_cast<char*>(h_pub_) + sizeof(Scal) * kMaxSys);
    std::memset(h_flags_, 0, sizeof(Scal) * kMaxSys * 4 + 256);
    h_blk_flag_ = reinterpret_cast<unsigned*>(reinterpret_cast<char*>(h_flags_) + sizeof(Scal) * kMaxSys * 4);
  }
}

void Engine::set_profiling(bool on) {
  profiling_ = on;
  for (auto& a : stat)
    for (auto& b : a) b = KernelStat{};
}

Engine::~Engine() {
  (void)hipStreamSynchronize(st_);
  for (hipEvent_t e : events_) (void)hipEventDestroy(e);
  for (System* s : slots_)
    if (s) remove(s);
  if (d_desc_) (void)hipFree(d_desc_);
  if (h_desc_) (void)hipHostFree(h_desc_);
  if (d_y_) (void)hipFree(d_y_);
  if (h_y_) (void)hipHostFree(h_y_);
  if (d_scal_) (void)hipFree(d_scal_);
  if (h_scal_) (void)hipHostFree(h_scal_);
  if (h_flags_) (void)hipHostFree(h_flags_);
  if (h_pub_) (void)hipHostFree(h_pub_);
}

bool Engine::idle() const {
  for (System* s : slots_)
    if (s && !s->done) return false;
  return true;
}

int Engine::count() const {
  int c = 0;
  for (System* s : slots_) c += s != nullptr;
  return c;
}

static bool is_fgmres(const hub_solve_opts& o) { return o.solver == HUB_FGMRES_MIXED; }

size_t Engine::workspace_bytes(const Geom& g, const hub_solve_opts& o) {
  const size_t n = (size_t)g.n;
  const size_t part = Pool::rounded((size_t)tile_geo(g, spt_of(g.n)).ntiles * (kMaxRed + 2) * sizeof(double));
  // vectors + the phase tables that `add` computes when the caller brings none
  // (FP64 phase n * 16; the mixed solver's float angle n * 4)
  if (!is_fgmres(o)) return 5 * Pool::rounded(n * 16) + part;
  const int m = o.restart_m;
  // small systems also keep the (cos, sin) table of the single-workgroup CG
  return (size_t)(m + 4) * Pool::rounded(n * 16) + (size_t)(m + 4 + (wg_of(g.n) ? 1 : 0)) * Pool::rounded(n * 8) +
         Pool::rounded(n * 4) + part;
}

Engine::AddResult Engine::add(System* s) {
  int slot = -1;
  for (int k = 0; k < kMaxSys; ++k)
    if (!slots_[k]) {
      slot = k;
      break;
    }
  if (slot < 0) {
    set_error("engine full");
    return ADD_NO_ROOM;
  }
  const size_t n = (size_t)s->g.n;
  SysDesc& d = s->desc;
  std::memset(&d, 0, sizeof(d));
  d.g = s->g;
  d.mu2 = s->mu2;
  d.phi = s->phi;
  d.spt = spt_of(s->g.n);
  const TileGeo tg = tile_geo(s->g, d.spt);
  d.tnb = tg.nb;
  d.tbsz = tg.bsz;
  d.tseg = tg.seg;
  d.ntiles = tg.ntiles;
  d.sc = d_scal_ + slot;
  auto get = [&](size_t bytes) -> void* {
    void* p = pool_->alloc(bytes, st_);
    if (p) s->owned.push_back(p);
    return p;
  };
  bool ok = true, hip_ok = true;
  d.part = (double*)get((size_t)d.ntiles * (kMaxRed + 2) * sizeof(double));
  ok = ok && d.part;
  if (ok) {
    d.part1 = d.part + (size_t)d.ntiles * kMaxRed;
    d.part2 = d.part1 + d.ntiles;
  }
  d.vec[S_B] = (void*)s->b;
  d.vec[S_X] = (void*)s->x;
  if (!is_fgmres(s->opts)) {
    for (int k : {(int)S_R, (int)S_P0, (int)S_P0 + 1, (int)S_U}) {
      d.vec[k] = get(n * 16);
      ok = ok && d.vec[k];
    }
  } else {
    const int m = s->opts.restart_m;
    for (int k : {(int)S_R, (int)S_U}) {
      d.vec[k] = get(n * 16);
      ok = ok && d.vec[k];
    }
    for (int k = 0; k <= m && ok; ++k) {
      d.vec[S_V0 + k] = get(n * 16);
      ok = ok && d.vec[S_V0 + k];
    }
    for (int k : {(int)S_R32, (int)S_P32, (int)S_P32 + 1, (int)S_U32}) {
      if (!ok) break;
      d.vec[k] = get(n * 8);
      ok = ok && d.vec[k];
    }
    for (int k = 0; k < m && ok; ++k) {
      d.vec[S_Z0 + k] = get(n * 8);
      ok = ok && d.vec[S_Z0 + k];
    }
  }
  // the phase e^{i phi} of the solver kernels (shared with other systems when the
  // caller precomputed it)
  const bool want32 = is_fgmres(s->opts);
  const bool wantcs = want32 && wg_of(s->g.n);
  if (ok && (!s->ph64 || (want32 && !s->ph32) || (wantcs && !s->cs32))) {
    double2* p64 = (double2*)get(n * 16);
    float* p32 = want32 ? (float*)get(n * 4) : nullptr;
    float2* pcs = wantcs ? (float2*)get(n * 8) : nullptr;
    ok = ok && p64 && (!want32 || p32) && (!wantcs || pcs);
    if (ok && launch_phase(s->phi, p64, p32, (int)n, st_, pcs) != hipSuccess) ok = hip_ok = false;
    if (ok) {
      s->ph64 = p64;
      s->ph32 = p32;
      s->cs32 = pcs;
    }
  }
  d.ph64 = s->ph64;
  d.ph32 = s->ph32;
  d.cs32 = s->cs32;
  if (!ok) {
    pool_->release_all(s->owned, st_);
    s->owned.clear();
    if (!hip_ok) set_error("phase launch failed");
    return hip_ok ? ADD_NO_ROOM : ADD_HIP;
  }
  s->slot = slot;
  s->wg = wantcs;
  s->phase = PH_NEW;
  s->done = false;
  s->info = hub_solve_info{};
  slots_[slot] = s;
  upload_desc(s);
  return ADD_OK;
}

void Engine::remove(System* s) {
  // drain blocks that still reference the system
  for (auto& q : inflight_) {
    bool refs = false;
    for (auto& b : q)
      for (System* x : b.v) refs = refs || x == s;
    if (!refs) continue;
    // an error here surfaces again at the next synchronising call of the stream
    for (auto& b : q) (void)finish_block(b);
    q.clear();
  }
  if (s->slot >= 0 && slots_[s->slot] == s) slots_[s->slot] = nullptr;
  pool_->release_all(s->owned, st_);
  s->owned.clear();
  s->slot = -1;
}

void Engine::upload_desc(System* s) {
  h_desc_[s->slot] = s->desc;
  desc_lo_ = std::min(desc_lo_, s->slot);
  desc_hi_ = std::max(desc_hi_, s->slot);
}

void Engine::upload_y(System* s, const std::vector<std::complex<double>>& y) {
  static_assert(sizeof(std::complex<double>) == 2 * sizeof(double), "complex layout");
  double* row = h_y_ + (size_t)s->slot * kYStride;
  for (size_t i = 0; i < y.size() && (int)i < kMaxRestart; ++i) {
    row[2 * i] = y[i].real();
    row[2 * i + 1] = y[i].imag();
  }
  y_lo_ = std::min(y_lo_, s->slot);
  y_hi_ = std::max(y_hi_, s->slot);
}

hipError_t Engine::flush_desc() {
  if (desc_hi_ < desc_lo_) return hipSuccess;
  const hipError_t e = hipMemcpyAsync(d_desc_ + desc_lo_, h_desc_ + desc_lo_, sizeof(SysDesc) * (desc_hi_ - desc_lo_ + 1),
                                      hipMemcpyHostToDevice, st_);
  desc_lo_ = kMaxSys;
  desc_hi_ = -1;
  return e;
}

hipError_t Engine::flush_y() {
  if (y_hi_ < y_lo_) return hipSuccess;
  const hipError_t e = hipMemcpyAsync(d_y_ + (size_t)y_lo_ * kYStride, h_y_ + (size_t)y_lo_ * kYStride,
                                      sizeof(double) * kYStride * (y_hi_ - y_lo_ + 1), hipMemcpyHostToDevice, st_);
  y_lo_ = kMaxSys;
  y_hi_ = -1;
  return e;
}

LaunchList Engine::one(System* s) const { return list(std::vector<System*>{s}); }

LaunchList Engine::list(const std::vector<System*>& v) const {
  LaunchList L;
  std::memset(&L, 0, sizeof(L));
  L.scal = d_scal_;
  L.nsys = (int)v.size();
  // every system of a list has the same tile class (callers group them)
  L.spt = v.empty() ? kSitesPerThread : v.front()->desc.spt;
  int acc = 0;
  for (int k = 0; k < L.nsys; ++k) {
    L.tile_begin[k] = acc;
    L.sys[k] = v[k]->slot;
    acc += v[k]->desc.ntiles;
  }
  L.tile_begin[L.nsys] = acc;
  for (int k = L.nsys + 1; k <= kMaxSys; ++k) L.tile_begin[k] = acc;
  L.total_tiles = acc;
  return L;
}

hipError_t Engine::read_scal(const std::vector<System*>& v) {
  int lo = kMaxSys, hi = -1;
  for (System* s : v) {
    lo = std::min(lo, s->slot);
    hi = std::max(hi, s->slot);
  }
  if (hi < lo) return hipSuccess;
  // A kernel writes the records and then a sequence number to host-coherent memory and
  // the host polls the number: about half the latency of a copy plus a stream
  // synchronisation.  hipStreamQuery bounds the wait; should the stream drain without
  // the number showing, the records are read through a copy instead.
  const int cnt = hi - lo + 1;
  const unsigned seq = ++pub_seq_;
  HUB_TRY(launch_publish(d_scal_ + lo, h_pub_ + lo, cnt, h_pub_flag_, seq, st_));
  for (unsigned spin = 1;; ++spin) {
    if (__atomic_load_n(h_pub_flag_, __ATOMIC_ACQUIRE) == seq) break;
    if ((spin & 255) == 0) {
      const hipError_t q = hipStreamQuery(st_);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) return q;
      if (__atomic_load_n(h_pub_flag_, __ATOMIC_ACQUIRE) == seq) break;
      HUB_TRY(hipMemcpyAsync(h_scal_ + lo, d_scal_ + lo, sizeof(Scal) * cnt, hipMemcpyDeviceToHost, st_));
      return hipStreamSynchronize(st_);
    }
  }
  std::memcpy(h_scal_ + lo, h_pub_ + lo, sizeof(Scal) * cnt);
  return hipSuccess;
}

void Engine::finish(System* s, hub_status st) {
  s->status = st;
  s->phase = PH_DONE;
  s->done = true;
  s->info.converged = st == HUB_OK ? 1 : 0;
}

// One host-side transition for a group of systems at the same phase (and, in
// FGMRES, the same Arnoldi step): one launch per kernel over the group's systems and
// one read-back for all of them (the per-system arithmetic is that of a system alone).
hipError_t Engine::group_phase(int phase, const std::vector<System*>& g) {
  const int j = g.front()->j;
  switch (phase) {
    case PH_NEW: {
      // the group shares the solver and whether x0 is used
      const hub_solve_opts& og = g.front()->opts;
      LaunchList L = list(g);
      if (!is_fgmres(og)) {
        // FP64 CG: r = b - A x (x = 0 or x0) and the CG start
        if (!og.use_x0) {
          for (size_t q = 0; q < g.size(); ++q) {
            L.pa[q] = 0.0;
            L.pr[q] = g[q]->opts.tol * g[q]->opts.tol;
            L.pi[q] = g[q]->opts.max_iter;
          }
          HUB_TRY(launch_cg_init_zero(d_desc_, L, RED_CG_SETUP, st_));
        } else {
          HUB_TRY(launch_multidot(d_desc_, L, S_B, S_B, 1, 0, st_));
          HUB_TRY(read_scal(g));
          for (size_t q = 0; q < g.size(); ++q) {
            System* s = g[q];
            s->bb = h_scal_[s->slot].red[0];
            L.pa[q] = s->opts.tol * s->opts.tol * s->bb;
            L.pr[q] = 0.0;
            L.pi[q] = s->opts.max_iter;
            s->info.applies++;
          }
          HUB_TRY(launch_normal_slot(d_desc_, L, S_X, false, S_B, S_R, RED_CG_SETUP, 1, st_));
        }
        for (System* s : g) {
          s->enq = 0;
          s->gen++;
          s->phase = PH_CG_ITER;
        }
        return hipSuccess;
      }
      // FGMRES: r = b (or b - A x0), |b|
      if (!og.use_x0) {
        HUB_TRY(launch_cg_init_zero(d_desc_, L, RED_STORE, st_));
      } else {
        HUB_TRY(launch_multidot(d_desc_, L, S_B, S_B, 1, 0, st_));
        HUB_TRY(launch_normal_slot(d_desc_, L, S_X, false, S_B, S_R, RED_STORE, 2, st_));
      }
      HUB_TRY(read_scal(g));
      std::vector<System*> run, zero;
      for (System* s : g) {
        const Scal& sc = h_scal_[s->slot];
        s->bb = sc.red[0];
        s->err = og.use_x0 ? std::sqrt(sc.red[2]) : std::sqrt(s->bb);
        if (og.use_x0) s->info.applies++;
        s->bnorm = std::sqrt(s->bb);
        if (!std::isfinite(s->bb) || !std::isfinite(s->err)) {
          // phi, b or the initial guess holds a non-finite value
          finish(s, HUB_ERR_ARG);
        } else if (s->bnorm == 0.0) {
          zero.push_back(s);
        } else if (s->err <= s->opts.tol * s->bnorm) {
          s->info.true_rel_resid = s->err / s->bnorm;
          finish(s, HUB_OK);
        } else {
          run.push_back(s);
        }
      }
      if (!zero.empty()) {
        // b = 0: x = 0 exactly
        HUB_TRY(launch_cg_init_zero(d_desc_, list(zero), RED_STORE, st_));
        for (System* s : zero) {
          s->info.true_rel_resid = 0.0;
          finish(s, HUB_OK);
        }
      }
      if (run.empty()) return hipSuccess;
      // initial single-precision solve on r (Algorithm A.1, first line)
      LaunchList R = list(run);
      for (size_t q = 0; q < run.size(); ++q) {
        const System* s = run[q];
        const hub_solve_opts& o = s->opts;
        const double tau = std::max(std::min(o.tol * o.inner_a * s->bnorm / s->err, 1.0), o.inner_floor);
        R.pa[q] = 1.0;
        R.pr[q] = tau * tau;
        R.pi[q] = o.inner_max_iter;
        R.pj[q] = S_Z0;
      }
      HUB_TRY(launch_prep_inner(d_desc_, R, S_R, -1, st_));
      for (System* s : run) {
        s->enq = 0;
        s->gen++;
        s->phase = PH_F_INNER;
        s->post = PH_F_POST_INIT;
      }
      return hipSuccess;
    }
    case PH_CG_CONFIRM: {
      // FP64 true residual of the CG iterate; restart the CG from x if it misses tol.
      // |b|^2 comes from the CG start, whose reduction is NaN when phi or b holds a
      // non-finite value: such systems stop here.
      std::vector<System*> ok;
      for (System* s : g) {
        if (!std::isfinite(s->bb))
          finish(s, HUB_ERR_ARG);
        else
          ok.push_back(s);
      }
      if (ok.empty()) return hipSuccess;
      return confirm(ok);
    }
    case PH_F_POST_INIT: {
      // x = z_0 (or x0 + z_0), r = b - A x, ERR = |r|
      for (System* s : g) upload_y(s, {std::complex<double>(1.0, 0.0)});
      HUB_TRY(flush_y());
      const LaunchList L = list(g);
      HUB_TRY(launch_xupdate(d_desc_, L, d_y_, 1, !g.front()->opts.use_x0, st_));
      HUB_TRY(launch_normal_slot(d_desc_, L, S_X, false, S_B, S_R, RED_STORE, 0, st_));
      HUB_TRY(read_scal(g));
      for (System* s : g) {
        const hub_solve_opts& o = s->opts;
        s->info.applies++;
        s->err = std::sqrt(h_scal_[s->slot].red[0]);
        s->info.true_rel_resid = s->err / s->bnorm;
        if (s->err <= o.tol * s->bnorm) {
          finish(s, HUB_OK);
          continue;
        }
        s->j = 0;
        s->wnorm = s->err;
        s->rnorm_cycle = s->err;
        s->H.assign((size_t)(o.restart_m + 1) * o.restart_m, std::complex<double>(0.0));
        s->phase = PH_F_ARNOLDI;
      }
      return hipSuccess;
    }
    case PH_F_ARNOLDI: {
      // v_j = w / |w|; z_j from the single-precision CG when TOL a |b| / ERR < 1, else z_j = v_j
      std::vector<System*> act;
      for (System* s : g) {
        if (s->err < s->opts.tol * s->bnorm || s->wnorm == 0.0 || !std::isfinite(s->wnorm))
          s->phase = PH_F_LSQ;
        else
          act.push_back(s);
      }
      if (act.empty()) return hipSuccess;
      LaunchList L = list(act);
      for (size_t q = 0; q < act.size(); ++q) {
        const System* s = act[q];
        const hub_solve_opts& o = s->opts;
        const double ratio = o.tol * o.inner_a * s->bnorm / s->err;
        L.pa[q] = 1.0 / s->wnorm;
        L.pj[q] = S_Z0 + j;
        if (ratio < 1.0) {
          const double tau = std::max(ratio, o.inner_floor);
          L.pr[q] = tau * tau;
          L.pi[q] = o.inner_max_iter;
        } else {
          L.pr[q] = 0.0;
          L.pi[q] = 0;
        }
      }
      HUB_TRY(launch_prep_inner(d_desc_, L, S_R, S_V0 + j, st_));
      for (size_t q = 0; q < act.size(); ++q) {
        System* s = act[q];
        if (L.pi[q] > 0) {
          s->enq = 0;
          s->gen++;
          s->phase = PH_F_INNER;
          s->post = PH_F_POST_ARNOLDI;
        } else {
          s->phase = PH_F_POST_ARNOLDI;
        }
      }
      return hipSuccess;
    }
    case PH_F_POST_ARNOLDI: {
      // w = A z_j, classical Gram-Schmidt against v_0 .. v_j, h_{j+1,j} = |w|, ERR *= |w|:
      // the smallest systems in one fused launch, the others on the tiled kernels
      std::vector<System*> gw, gt;
      for (System* s : g) (arn_wg_of(s->g.n) ? gw : gt).push_back(s);
      if (!gt.empty()) {
        const LaunchList L = list(gt);
        HUB_TRY(launch_normal_slot(d_desc_, L, S_Z0 + j, true, -1, S_R, RED_NONE, 0, st_));
        HUB_TRY(launch_multidot(d_desc_, L, S_R, S_V0, j + 1, 0, st_));
        HUB_TRY(launch_cgs(d_desc_, L, S_R, S_V0, j + 1, 0, 2 * (j + 1), st_));
      }
      if (!gw.empty()) {
        WgList W;
        std::memset(&W, 0, sizeof(W));
        W.scal = d_scal_;
        W.nsys = (int)gw.size();
        for (size_t q = 0; q < gw.size(); ++q) {
          W.sys[q] = gw[q]->slot;
          W.nmax = std::max(W.nmax, gw[q]->g.n);
        }
        HUB_TRY(launch_arnoldi_wg(d_desc_, W, j, st_));
      }
      HUB_TRY(read_scal(g));
      for (System* s : g) {
        const int m = s->opts.restart_m;
        s->info.applies++;
        const Scal& sc = h_scal_[s->slot];
        for (int i = 0; i <= j; ++i) s->H[(size_t)j * (m + 1) + i] = {sc.red[2 * i], sc.red[2 * i + 1]};
        const double hn = std::sqrt(std::max(sc.red[2 * (j + 1)], 0.0));
        s->H[(size_t)j * (m + 1) + j + 1] = hn;
        s->wnorm = hn;
        // ERR: the residual of the best iterate of the cycle so far, the least-squares
        // residual of the Arnoldi relation (Algorithm A.1's ERR * |w| is this quantity
        // while every step's inner solve meets its tolerance, and not after an
        // unpreconditioned step, where it ends cycles that have not converged)
        double res = s->err;
        (void)hessenberg_lsq(s->H, m + 1, j + 1, s->rnorm_cycle, &res);
        s->err = res;
        s->j = j + 1;
        s->phase = (s->j == m) ? PH_F_LSQ : PH_F_ARNOLDI;
      }
      return hipSuccess;
    }
    case PH_F_LSQ: {
      // y = argmin |(|r|, 0, ..) - H y|, x += sum y_i z_i, true residual, restart or stop
      const int k = j;
      const LaunchList L = list(g);
      if (k > 0) {
        for (System* s : g) upload_y(s, hessenberg_lsq(s->H, s->opts.restart_m + 1, k, s->rnorm_cycle));
        HUB_TRY(flush_y());
        HUB_TRY(launch_xupdate(d_desc_, L, d_y_, k, false, st_));
      }
      HUB_TRY(launch_normal_slot(d_desc_, L, S_X, false, S_B, S_R, RED_STORE, 0, st_));
      HUB_TRY(read_scal(g));
      for (System* s : g) {
        const hub_solve_opts& o = s->opts;
        s->info.applies++;
        s->cycles++;
        s->info.outer_iters = s->cycles;
        s->err = std::sqrt(h_scal_[s->slot].red[0]);
        s->info.true_rel_resid = s->err / s->bnorm;
        if (s->err <= o.tol * s->bnorm) {
          finish(s, HUB_OK);
        } else if (s->cycles >= o.max_iter || !std::isfinite(s->err) || k == 0) {
          finish(s, HUB_ERR_NOCONV);
        } else {
          s->j = 0;
          s->wnorm = s->err;
          s->rnorm_cycle = s->err;
          std::fill(s->H.begin(), s->H.end(), std::complex<double>(0.0));
          s->phase = PH_F_ARNOLDI;
        }
      }
      return hipSuccess;
    }
    default:
      return hipSuccess;
  }
}

// FP64 true residual of the CG iterates of g (finite |b|^2); restart a CG from x where it
// misses tol, or stop the system.
hipError_t Engine::confirm(const std::vector<System*>& g) {
  LaunchList L = list(g);
  for (size_t q = 0; q < g.size(); ++q) {
    const System* s = g[q];
    L.pa[q] = s->opts.tol * s->opts.tol * s->bb;
    L.pr[q] = 0.0;
    L.pi[q] = std::max(1, s->opts.max_iter - s->cg_total);
  }
  HUB_TRY(launch_normal_slot(d_desc_, L, S_X, false, S_B, S_R, RED_CG_SETUP, 1, st_));
  HUB_TRY(read_scal(g));
  for (System* s : g) {
    const hub_solve_opts& o = s->opts;
    s->info.applies++;
    const double rr = h_scal_[s->slot].red[1];
    s->info.true_rel_resid = s->bb > 0 ? std::sqrt(rr / s->bb) : 0.0;
    if (s->info.true_rel_resid <= o.tol) {
      finish(s, HUB_OK);
    } else if (!std::isfinite(rr) && s->cg_total == 0) {
      // r = b - A x0 is not finite before any iteration: phi or x0 is not finite
      finish(s, HUB_ERR_ARG);
    } else if (s->cg_total >= o.max_iter || !std::isfinite(rr)) {
      finish(s, HUB_ERR_NOCONV);
    } else {
      s->info.outer_iters++;
      s->enq = 0;
      s->gen++;
      s->phase = PH_CG_ITER;
    }
  }
  return hipSuccess;
}

// Enqueue one block of CG iterations over every system that is iterating in the
// given precision, followed by an asynchronous read-back of their flags.
hipError_t Engine::launch_block(bool single, bool& launched) {
  launched = false;
  std::vector<System*> v;
  int k = 1 << 30;
  bool any_tiled = false;
  for (System* s : slots_) {
    if (!s || s->done) continue;
    if ((single && s->phase == PH_F_INNER) || (!single && s->phase == PH_CG_ITER)) {
      v.push_back(s);
      any_tiled = any_tiled || !(single && s->wg);
      int ks = std::max(1, s->opts.check_every);
      // near the iteration count of the system's previous CG run, enqueue short
      // blocks: launches after convergence return at once but still cost a launch
      if (s->pred > 0 && s->enq + ks > s->pred - kTailBlock) ks = std::min(ks, kTailBlock);
      k = std::min(k, ks);
    }
  }
  if (v.empty()) return hipSuccess;
  // Only single-workgroup systems iterating: their kernel stops by itself within a
  // block, so long blocks cost nothing after convergence and save the per-block
  // flag read-backs.
  if (!any_tiled) k = std::max(k, kWgBlockIters);
  // small systems run the whole block in one single-workgroup launch
  std::vector<System*> wgs;
  for (System* s : v)
    if (single && s->wg) wgs.push_back(s);
  // the others by the tile size of their CG stages: one launch per size class
  std::vector<System*> ordered;
  std::vector<int> cls_spt, cls_end;
  for (int spt : {(int)kSitesPerThread, (int)kSmallSpt}) {
    for (System* s : v)
      if (!(single && s->wg) && s->desc.spt == spt) ordered.push_back(s);
    if (!ordered.empty() && (cls_end.empty() || (int)ordered.size() > cls_end.back())) {
      cls_spt.push_back(spt);
      cls_end.push_back((int)ordered.size());
    }
    if (kSmallSpt == kSitesPerThread) break;
  }
  const int ntile = (int)ordered.size();
  v = ordered;
  const int ncls = (int)cls_spt.size();
  Block b;
  b.single = single;
  b.k = k;
  b.v = v;
  b.v.insert(b.v.end(), wgs.begin(), wgs.end());
  b.nwg = (int)wgs.size();
  b.cls_end = cls_end;
  for (System* s : b.v) b.gen.push_back(s->gen);
  b.buf = next_buf_[single ? 1 : 0];
  next_buf_[single ? 1 : 0] ^= 1;
  std::vector<LaunchList> Ls;
  for (int c = 0; c < ncls; ++c) {
    const int q0 = c == 0 ? 0 : cls_end[c - 1];
    std::vector<System*> vc(v.begin() + q0, v.begin() + cls_end[c]);
    LaunchList L = list(vc);
    // The solution slot of the initial single-precision solve is S_Z0 (j = 0 then).
    for (size_t q = 0; q < vc.size(); ++q) L.pi[q] = single ? S_Z0 + vc[q]->j : S_X;
    Ls.push_back(L);
  }
  auto take_event = [&](std::vector<hipEvent_t>& dst) -> hipError_t {
    if (events_.empty()) {
      hipEvent_t ev;
      HUB_TRY(hipEventCreate(&ev));
      events_.push_back(ev);
    }
    dst.push_back(events_.back());
    events_.pop_back();
    return hipSuccess;
  };
  if (profiling_) {
    for (int e = 0; e < 4 * k * ncls; ++e) HUB_TRY(take_event(b.kev));
    if (b.nwg > 0) {
      HUB_TRY(take_event(b.wgev));
      HUB_TRY(take_event(b.wgev));
    }
  }
  if (b.nwg > 0) {
    WgList W;
    std::memset(&W, 0, sizeof(W));
    W.scal = d_scal_;
    W.nsys = b.nwg;
    for (int q = 0; q < b.nwg; ++q) {
      System* s = wgs[q];
      W.nmax = std::max(W.nmax, s->g.n);
      W.sys[q] = s->slot;
      W.pi[q] = single ? S_Z0 + s->j : S_X;
      W.it[q] = s->enq;
      s->enq += k;
    }
    HUB_TRY(launch_cg_wg(d_desc_, W, k, st_, profiling_ ? b.wgev[0] : nullptr, profiling_ ? b.wgev[1] : nullptr));
  }
  for (int it = 0; it < k && ntile > 0; ++it) {
    std::vector<int> its(ntile);
    for (int q = 0; q < ntile; ++q) its[q] = v[q]->enq++;
    for (int c = 0; c < ncls; ++c) {
      const int q0 = c == 0 ? 0 : cls_end[c - 1];
      for (int q = q0; q < cls_end[c]; ++q) Ls[c].it[q - q0] = its[q];
    }
    if (!profiling_) {
      for (int c = 0; c < ncls; ++c) HUB_TRY(launch_cg_iter(d_desc_, Ls[c], single, st_));
      continue;
    }
    b.its.push_back(its);
    for (int stage = 1; stage <= 2; ++stage)
      for (int c = 0; c < ncls; ++c) {
        const int e = 4 * (it * ncls + c) + 2 * (stage - 1);
        HUB_TRY(launch_cg_stage(d_desc_, Ls[c], single, stage, st_, b.kev[e], b.kev[e + 1]));
      }
  }
  int lo = kMaxSys, hi = -1;
  for (System* s : b.v) {
    lo = std::min(lo, s->slot);
    hi = std::max(hi, s->slot);
  }
  // The block's flags go to host-coherent memory through a kernel that then writes the
  // block's sequence number (k_publish): unlike a device-to-host copy followed by an
  // event, it adds no barrier packet, so the next block's kernels follow at once.
  Scal* dst = h_flags_ + (size_t)((single ? 2 : 0) + b.buf) * kMaxSys;
  b.seq = ++blk_seq_;
  HUB_TRY(launch_publish(d_scal_ + lo, dst + lo, hi - lo + 1, h_blk_flag_, b.seq, st_));
  inflight_[single ? 1 : 0].push_back(std::move(b));
  launched = true;
  return hipSuccess;
}

// Wait until the flags of the block with sequence number seq are in host memory.  Blocks
// publish in stream order, so a later number showing implies this block's records.  The
// spin checks the stream every so often: an error ends it, and a drained stream without
// the number (which a completed publish kernel rules out) is reported as an error.
hipError_t Engine::wait_block(unsigned seq) {
  for (unsigned spin = 1;; ++spin) {
    if ((int)(__atomic_load_n(h_blk_flag_, __ATOMIC_ACQUIRE) - seq) >= 0) return hipSuccess;
    if ((spin & 255) == 0) {
      const hipError_t q = hipStreamQuery(st_);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) return q;
      if ((int)(__atomic_load_n(h_blk_flag_, __ATOMIC_ACQUIRE) - seq) >= 0) return hipSuccess;
      set_error("CG block flags not published");
      return hipErrorUnknown;
    }
  }
}

// Wait for a block's flags and move the systems that stopped iterating on.
hipError_t Engine::finish_block(Block& b) {
  HUB_TRY(wait_block(b.seq));
  const bool single = b.single;
  const Scal* flags = h_flags_ + (size_t)((single ? 2 : 0) + b.buf) * kMaxSys;
  if (profiling_ && !b.kev.empty()) {
    // A system did work in the launch of iteration `it` iff it < its final count
    // (or it is still iterating).
    const int ncls = (int)b.cls_end.size();
    for (int it = 0; it < b.k; ++it) {
      for (int c = 0; c < ncls; ++c) {
        const int q0 = c == 0 ? 0 : b.cls_end[c - 1];
        for (int stage = 0; stage < 2; ++stage) {
          double bytes = 0.0;
          for (int q = q0; q < b.cls_end[c]; ++q) {
            const Scal& sc = flags[b.v[q]->slot];
            const int its = b.its[it][q];
            if (sc.active || its < sc.iters) bytes += (double)b.v[q]->g.n * cg_bytes(single, stage + 1, its);
          }
          const int e = 4 * (it * ncls + c) + 2 * stage;
          float ms = 0.0f;
          HUB_TRY(hipEventElapsedTime(&ms, b.kev[e], b.kev[e + 1]));
          KernelStat& ks = stat[single ? 1 : 0][stage];
          ks.launches++;
          ks.ms += ms;
          ks.bytes += bytes;
        }
      }
    }
  }
  if (profiling_ && b.wgev.size() == 2) {
    float ms = 0.0f;
    HUB_TRY(hipEventElapsedTime(&ms, b.wgev[0], b.wgev[1]));
    KernelStat& ks = stat[single ? 1 : 0][2];
    ks.launches++;
    ks.ms += ms;
  }
  for (hipEvent_t e : b.kev) events_.push_back(e);
  for (hipEvent_t e : b.wgev) events_.push_back(e);
  b.kev.clear();
  b.wgev.clear();
  for (size_t q = 0; q < b.v.size(); ++q) {
    System* s = b.v[q];
    const bool want = single ? (s->phase == PH_F_INNER) : (s->phase == PH_CG_ITER);
    // skip a system that an earlier block already moved on (its flags here
    // belong to a finished CG run)
    if (s->done || !want || s->gen != b.gen[q]) continue;
    const Scal& sc = flags[s->slot];
    if (sc.active) continue;
    s->pred = sc.iters;
    if (single) {
      s->info.inner_iters += sc.iters;
      s->phase = s->post;
    } else {
      s->cg_total += sc.iters;
      s->info.inner_iters = s->cg_total;
      if (s->bb < 0) s->bb = sc.red[0];
      s->phase = PH_CG_CONFIRM;
    }
  }
  return hipSuccess;
}

hipError_t Engine::step() {
  // 0. descriptors of systems added since the last step
  HUB_TRY(flush_desc());
  // 1. keep the GPU busy: enqueue the next block for every system still iterating
  //    (speculatively: a system that converged in the block still in flight runs
  //    empty launches, which return at once)
  bool launched[2] = {false, false};
  HUB_TRY(launch_block(false, launched[0]));
  HUB_TRY(launch_block(true, launched[1]));
  // 2. read back older blocks: keep one in flight while that precision iterates
  for (int k = 0; k < 2; ++k) {
    auto& q = inflight_[k];
    const size_t keep = launched[k] ? 1 : 0;
    while (q.size() > keep) {
      HUB_TRY(finish_block(q.front()));
      q.erase(q.begin());
    }
  }
  // 3. host-side phases of the systems that are not iterating, in groups of systems
  //    at the same phase (and Arnoldi step)
  bool progressed = true;
  while (progressed) {
    progressed = false;
    for (int ph : {(int)PH_NEW, (int)PH_CG_CONFIRM, (int)PH_F_POST_INIT, (int)PH_F_LSQ, (int)PH_F_POST_ARNOLDI,
                   (int)PH_F_ARNOLDI}) {
      // key: Arnoldi step, solver, whether x0 is used (the start's and the first
      // update's kernels depend on them) and tile class (one per launch)
      std::map<int, std::vector<System*>> groups;
      for (System* s : slots_)
        if (s && !s->done && s->phase == ph)
          groups[8 * s->j + (s->desc.spt == kSmallSpt ? 4 : 0) + (is_fgmres(s->opts) ? 2 : 0) +
                 (s->opts.use_x0 ? 1 : 0)]
              .push_back(s);
      for (auto& kv : groups) {
        HUB_TRY(group_phase(ph, kv.second));
        progressed = true;
        for (System* s : kv.second)
          if (s->done && s->on_done) s->on_done(s);
      }
    }
    bool all_wait = true;
    for (System* s : slots_)
      if (s && !s->done && s->phase != PH_F_INNER && s->phase != PH_CG_ITER) all_wait = false;
    if (all_wait) break;
  }
  return hipSuccess;
}

}  // namespace hub

namespace hub {

hipError_t Engine::finalize(System* s, const double2* chi, double* dSdphi, double* S) {
  const Geom& g = s->g;
  double2* xi = (double2*)s->desc.vec[S_U];
  HUB_TRY(launch_dot_re(g, chi, s->x, 1, s->desc.part, &d_scal_[s->slot].red[kMaxRed - 1], st_));
  if (dSdphi) {
    HUB_TRY(launch_apply(g, s->phi, s->x, xi, 1, true, st_));
    HUB_TRY(launch_force(g, s->phi, s->x, xi, 1.0, 0, dSdphi, 1, st_));
  }
  HUB_TRY(read_scal({s}));
  *S = h_scal_[s->slot].red[kMaxRed - 1];
  return hipSuccess;
}

}  // namespace hub
