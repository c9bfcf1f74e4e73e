// The C ABI of libhub (include/hub.h): argument checking, the context, the
// synchronous calls and the serving thread behind hub_submit / hub_poll.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <thread>

#include "hub.h"
#include "hub_engine.h"
#include "hub_md.h"

using namespace hub;

namespace {

hub_status fail(hub_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

hub_status hip_fail(hipError_t e, const char* where) {
  return fail(HUB_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HUB_HIP(expr, where)                       \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

bool is_finite(double v) { return std::isfinite(v); }

hub_status check_lattice(const hub_lattice* lat) {
  if (!lat) return fail(HUB_ERR_ARG, "lattice is NULL");
  if (lat->L1 < 1 || lat->L2 < 1 || lat->Nt < 1)
    return fail(HUB_ERR_ARG, "lattice extents must be >= 1");
  if (lat->reserved != 0) return fail(HUB_ERR_ARG, "hub_lattice.reserved must be 0");
  const long long n = 2LL * lat->L1 * lat->L2 * lat->Nt;
  if (n > (1LL << 30)) return fail(HUB_ERR_ARG, "lattice too large (2*L1*L2*Nt > 2^30)");
  if (!is_finite(lat->kappa_t) || !is_finite(lat->ms_t)) return fail(HUB_ERR_ARG, "couplings must be finite");
  return HUB_OK;
}

hub_status check_batch(int32_t batch) {
  if (batch < 1 || batch > HUB_MAX_BATCH) return fail(HUB_ERR_ARG, "batch must be in [1, HUB_MAX_BATCH]");
  return HUB_OK;
}

hub_status check_opts(const hub_solve_opts& o) {
  if (o.solver != HUB_CG_FP64 && o.solver != HUB_FGMRES_MIXED) return fail(HUB_ERR_ARG, "unknown solver");
  if (!is_finite(o.tol) || o.tol <= 0.0 || o.tol >= 1.0) return fail(HUB_ERR_ARG, "tol must be in (0, 1)");
  if (o.max_iter < 1) return fail(HUB_ERR_ARG, "max_iter must be >= 1");
  if (o.restart_m < 1 || o.restart_m > HUB_MAX_RESTART) return fail(HUB_ERR_ARG, "restart_m out of range");
  if (o.inner_max_iter < 1) return fail(HUB_ERR_ARG, "inner_max_iter must be >= 1");
  if (!is_finite(o.inner_a) || o.inner_a <= 0.0) return fail(HUB_ERR_ARG, "inner_a must be > 0");
  if (!is_finite(o.inner_floor) || o.inner_floor <= 0.0 || o.inner_floor >= 1.0)
    return fail(HUB_ERR_ARG, "inner_floor must be in (0, 1)");
  if (o.check_every < 1) return fail(HUB_ERR_ARG, "check_every must be >= 1");
  if (o.use_x0 != 0 && o.use_x0 != 1) return fail(HUB_ERR_ARG, "use_x0 must be 0 or 1");
  return HUB_OK;
}

static_assert(sizeof(hub_c128) == sizeof(double2), "hub_c128 layout");
static_assert(HUB_MAX_BATCH == kMaxSys, "batch limit");
static_assert(HUB_MAX_RESTART == kMaxRestart, "restart limit");
static_assert(HUB_MAX_HB_MASSES + 1 == kMaxLevels, "Hasenbusch levels");
static_assert(HUB_MAX_SHIFTS == kMsMax + 1, "multi-shift systems");
static_assert(HUB_MAX_HB_MASSES + 1 <= kMaxSys, "one batched solve per term");
static_assert(sizeof(hub_hmc_params) == 232 && sizeof(hub_md_op) == 152 && sizeof(hub_hmc_info) == 120,
              "HMC struct layouts");

// One served request.
struct Ticket {
  hub_request req;
  System sys;
  std::atomic<int> state{0};  // 0 queued, 1 running, 2 done
  hub_solve_info info{};
};

class Server;

}  // namespace

struct hub_ctx {
  int device = 0;
  std::unique_ptr<Pool> pool;
  std::mutex mu;  // serialises the synchronous calls
  std::map<hipStream_t, std::unique_ptr<Engine>> engines;
  std::unique_ptr<Server> server;
  std::mutex server_mu;
  bool profiling = false;
};

namespace {

// Continuous batching: admits queued requests whenever an engine slot and their
// workspace fit, and advances all admitted requests together.
class Server {
 public:
  explicit Server(hub_ctx* ctx) : ctx_(ctx) {
    hipSetDevice(ctx->device);
    hipStreamCreateWithFlags(&st_, hipStreamNonBlocking);
    engine_.reset(new Engine(ctx->pool.get(), st_));
    thread_ = std::thread([this] { run(); });
  }
  ~Server() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    thread_.join();
    engine_.reset();
    hipStreamDestroy(st_);
  }

  hub_status submit(const hub_request& r, uint64_t* ticket) {
    auto t = std::make_shared<Ticket>();
    t->req = r;
    System& s = t->sys;
    s.g = make_geom(r.lat);
    s.mu2 = r.mu2;
    s.phi = r.phi;
    s.b = (const double2*)r.chi;
    s.x = (double2*)r.x_out;
    s.opts = r.opts;
    if (Engine::workspace_bytes(s.g, s.opts) > ctx_->pool->budget())
      return fail(HUB_ERR_BUSY, "request workspace exceeds the serving budget");
    std::lock_guard<std::mutex> lk(mu_);
    const uint64_t id = ++next_;
    tickets_[id] = t;
    queue_.push_back(id);
    *ticket = id;
    cv_.notify_all();
    return HUB_OK;
  }

  hub_status poll(uint64_t id, int32_t* done, hub_solve_info* info) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = tickets_.find(id);
    if (it == tickets_.end()) return fail(HUB_ERR_NOTFOUND, "unknown ticket");
    if (it->second->state.load() != 2) {
      *done = 0;
      return HUB_OK;
    }
    *done = 1;
    if (info) *info = it->second->info;
    tickets_.erase(it);
    return HUB_OK;
  }

 private:
  void run() {
    hipSetDevice(ctx_->device);
    for (;;) {
      std::vector<uint64_t> admit;
      {
        std::unique_lock<std::mutex> lk(mu_);
        if (queue_.empty() && engine_->count() == 0) {
          if (stop_) return;
          cv_.wait_for(lk, std::chrono::milliseconds(5));
          continue;
        }
        // admit in arrival order while engine slots allow
        while (!queue_.empty() && engine_->count() + (int)admit.size() < kMaxSys) {
          admit.push_back(queue_.front());
          queue_.pop_front();
        }
      }
      std::vector<uint64_t> back;
      for (uint64_t id : admit) {
        if (!back.empty()) {
          back.push_back(id);
          continue;
        }
        std::shared_ptr<Ticket> t;
        {
          std::lock_guard<std::mutex> lk(mu_);
          t = tickets_[id];
        }
        System& s = t->sys;
        Ticket* tp = t.get();
        s.on_done = [this, tp](System* sp) { complete(tp, sp); };
        if (!engine_->add(&s)) {
          back.push_back(id);  // retried once running requests release workspace
          continue;
        }
        t->state = 1;
        running_.push_back(t);
      }
      if (!back.empty()) {
        std::lock_guard<std::mutex> lk(mu_);
        for (auto it = back.rbegin(); it != back.rend(); ++it) queue_.push_front(*it);
      }
      if (engine_->count() == 0) continue;
      if (engine_->step() != hipSuccess) {
        // a HIP failure: fail every running request
        for (auto& t : running_) {
          t->sys.status = HUB_ERR_HIP;
          t->info = t->sys.info;
          t->info.converged = 0;
          engine_->remove(&t->sys);
          t->state = 2;
        }
        running_.clear();
      }
      running_.erase(std::remove_if(running_.begin(), running_.end(),
                                    [](const std::shared_ptr<Ticket>& t) { return t->state.load() == 2; }),
                     running_.end());
    }
  }

  void complete(Ticket* t, System* s) {
    double S = 0.0;
    const hub_request& r = t->req;
    if (engine_->finalize(s, (const double2*)r.chi, r.dSdphi_out, &S) != hipSuccess) s->info.converged = 0;
    if (r.S_out) *r.S_out = S;
    t->info = s->info;
    engine_->remove(s);
    t->state = 2;
  }

  hub_ctx* ctx_;
  hipStream_t st_ = nullptr;
  std::unique_ptr<Engine> engine_;
  std::thread thread_;
  std::mutex mu_;
  std::condition_variable cv_;
  bool stop_ = false;
  uint64_t next_ = 0;
  std::map<uint64_t, std::shared_ptr<Ticket>> tickets_;
  std::deque<uint64_t> queue_;
  std::vector<std::shared_ptr<Ticket>> running_;
};

Engine* engine_for(hub_ctx* ctx, hipStream_t st) {
  auto it = ctx->engines.find(st);
  if (it != ctx->engines.end()) return it->second.get();
  Engine* e = new Engine(ctx->pool.get(), st);
  e->set_profiling(ctx->profiling);
  ctx->engines[st].reset(e);
  return e;
}

}  // namespace

extern "C" {

const char* hub_last_error(void) { return get_error(); }

void hub_default_opts(hub_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->solver = HUB_CG_FP64;
  o->max_iter = 20000;
  o->restart_m = 10;
  o->inner_max_iter = 4000;
  o->tol = 1e-10;
  o->inner_a = 5.0;
  o->inner_floor = 1e-5;
  o->use_x0 = 0;
  o->check_every = 16;
}

hub_status hub_create(hub_ctx** ctx, int device, size_t hbm_budget_bytes) {
  set_error("");
  if (!ctx) return fail(HUB_ERR_ARG, "ctx is NULL");
  *ctx = nullptr;
  int ndev = 0;
  HUB_HIP(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
  if (device < 0 || device >= ndev) return fail(HUB_ERR_ARG, "no such device");
  HUB_HIP(hipSetDevice(device), "hipSetDevice");
  size_t freeb = 0, total = 0;
  HUB_HIP(hipMemGetInfo(&freeb, &total), "hipMemGetInfo");
  hub_ctx* c = new hub_ctx;
  c->device = device;
  c->pool.reset(new Pool(device, hbm_budget_bytes ? hbm_budget_bytes : freeb / 4 * 3));
  *ctx = c;
  return HUB_OK;
}

hub_status hub_destroy(hub_ctx* ctx) {
  if (!ctx) return fail(HUB_ERR_ARG, "ctx is NULL");
  hipSetDevice(ctx->device);
  {
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    ctx->server.reset();
  }
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->engines.clear();
  }
  ctx->pool.reset();
  delete ctx;
  return HUB_OK;
}

static hub_status apply_common(hub_ctx* ctx, const hub_lattice* lat, const double* phi, const hub_c128* x,
                               hub_c128* y, int32_t batch, hipStream_t st, bool dag) {
  set_error("");
  if (!ctx) return fail(HUB_ERR_ARG, "ctx is NULL");
  hub_status s = check_lattice(lat);
  if (s) return s;
  if ((s = check_batch(batch))) return s;
  if (!phi || !x || !y) return fail(HUB_ERR_ARG, "NULL buffer");
  if ((const void*)x == (const void*)y) return fail(HUB_ERR_ARG, "x and y must not overlap");
  HUB_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  const Geom g = make_geom(*lat);
  HUB_HIP(launch_apply(g, phi, (const double2*)x, (double2*)y, batch, dag, st), "apply launch");
  return HUB_OK;
}

hub_status hub_apply_M(hub_ctx* ctx, const hub_lattice* lat, const double* phi, const hub_c128* x, hub_c128* y,
                       int32_t batch, hipStream_t stream) {
  return apply_common(ctx, lat, phi, x, y, batch, stream, false);
}

hub_status hub_apply_Mdag(hub_ctx* ctx, const hub_lattice* lat, const double* phi, const hub_c128* x, hub_c128* y,
                          int32_t batch, hipStream_t stream) {
  return apply_common(ctx, lat, phi, x, y, batch, stream, true);
}

hub_status hub_apply_normal(hub_ctx* ctx, const hub_lattice* lat, const double* phi, const double* mu2,
                            const hub_c128* x, hub_c128* y, int32_t batch, hipStream_t stream) {
  set_error("");
  if (!ctx) return fail(HUB_ERR_ARG, "ctx is NULL");
  hub_status s = check_lattice(lat);
  if (s) return s;
  if ((s = check_batch(batch))) return s;
  if (!phi || !x || !y || !mu2) return fail(HUB_ERR_ARG, "NULL buffer");
  if ((const void*)x == (const void*)y) return fail(HUB_ERR_ARG, "x and y must not overlap");
  double m2[kMaxSys] = {0};
  for (int b = 0; b < batch; ++b) {
    if (!is_finite(mu2[b]) || mu2[b] < 0) return fail(HUB_ERR_ARG, "mu2 must be finite and >= 0");
    m2[b] = mu2[b];
  }
  HUB_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  const Geom g = make_geom(*lat);
  void* u = ctx->pool->alloc((size_t)batch * g.n * 16, stream);
  if (!u) return HUB_ERR_OOM;
  hipError_t e = launch_apply(g, phi, (const double2*)x, (double2*)u, batch, true, stream);
  if (e == hipSuccess)
    e = launch_normal2(g, phi, m2, (const double2*)u, (const double2*)x, (double2*)y, batch, stream);
  ctx->pool->release(u, stream);
  if (e != hipSuccess) return hip_fail(e, "normal operator launch");
  return HUB_OK;
}

}  // extern "C"

namespace {

// Solves the prepared systems (each with its own geometry, shift, right-hand side
// and solution buffer; one phi) on the stream's engine, then synchronises the
// stream.  The caller holds ctx->mu and has set the device.  Per-system results are
// in sys[k].info and sys[k].status; the return value is the first failure
// (HUB_ERR_NOCONV if a system stopped at its iteration limit).
hub_status run_solves(hub_ctx* ctx, std::vector<System>& sys, const double* phi, const hub_solve_opts& o,
                      hipStream_t stream) {
  Engine* eng = engine_for(ctx, stream);
  const int n = sys.empty() ? 0 : sys[0].g.n;
  float* phi32 = nullptr;
  if (o.solver == HUB_FGMRES_MIXED) {
    phi32 = (float*)ctx->pool->alloc((size_t)n * 4, stream);
    if (!phi32) return fail(HUB_ERR_OOM, "workspace for phi in single precision");
    HUB_HIP(launch_phi_to_f32(phi, phi32, n, stream), "phi conversion");
  }
  hub_status result = HUB_OK;
  size_t added = 0;
  for (System& sy : sys) {
    sy.phi = phi;
    sy.phi32 = phi32;
    sy.opts = o;
    if (!eng->add(&sy)) {
      result = fail(HUB_ERR_OOM, "solver workspace");
      break;
    }
    ++added;
  }
  if (result == HUB_OK) {
    for (;;) {
      hipError_t e = eng->step();
      if (e != hipSuccess) {
        result = hip_fail(e, "solve");
        break;
      }
      bool all = true;
      for (const System& sy : sys) all = all && sy.done;
      if (all) break;
    }
  }
  for (size_t k = 0; k < added; ++k) eng->remove(&sys[k]);
  if (phi32) ctx->pool->release(phi32, stream);
  hipError_t e = hipStreamSynchronize(stream);
  if (result != HUB_OK) return result;
  if (e != hipSuccess) return hip_fail(e, "solve");
  for (const System& sy : sys)
    if (sy.status != HUB_OK && result == HUB_OK) result = sy.status;
  if (result == HUB_ERR_NOCONV) set_error("iteration limit reached before the tolerance");
  return result;
}

}  // namespace

extern "C" {

hub_status hub_solve(hub_ctx* ctx, const hub_lattice* lat, const double* phi, const double* mu2, int32_t batch,
                     const hub_c128* b, hub_c128* x, const hub_solve_opts* opts, hub_solve_info* info,
                     hipStream_t stream) {
  set_error("");
  if (!ctx) return fail(HUB_ERR_ARG, "ctx is NULL");
  hub_status s = check_lattice(lat);
  if (s) return s;
  if ((s = check_batch(batch))) return s;
  if (!phi || !b || !x || !mu2 || !info) return fail(HUB_ERR_ARG, "NULL buffer");
  hub_solve_opts o;
  hub_default_opts(&o);
  if (opts) o = *opts;
  if ((s = check_opts(o))) return s;
  for (int k = 0; k < batch; ++k)
    if (!is_finite(mu2[k]) || mu2[k] < 0) return fail(HUB_ERR_ARG, "mu2 must be finite and >= 0");
  std::lock_guard<std::mutex> lk(ctx->mu);
  HUB_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  const Geom g = make_geom(*lat);
  std::vector<System> sys((size_t)batch);
  for (int k = 0; k < batch; ++k) {
    sys[k].g = g;
    sys[k].mu2 = mu2[k];
    sys[k].b = (const double2*)(b + (size_t)k * g.n);
    sys[k].x = (double2*)(x + (size_t)k * g.n);
  }
  const hub_status result = run_solves(ctx, sys, phi, o, stream);
  if (result != HUB_OK && result != HUB_ERR_NOCONV) return result;
  for (int k = 0; k < batch; ++k) info[k] = sys[k].info;
  return result;
}

hub_status hub_force(hub_ctx* ctx, const hub_lattice* lat, const double* phi, const hub_c128* eta,
                     const hub_c128* xi, double scale, int32_t accumulate, double* dSdphi, int32_t batch,
                     hipStream_t stream) {
  set_error("");
  if (!ctx) return fail(HUB_ERR_ARG, "ctx is NULL");
  hub_status s = check_lattice(lat);
  if (s) return s;
  if ((s = check_batch(batch))) return s;
  if (!phi || !eta || !dSdphi) return fail(HUB_ERR_ARG, "NULL buffer");
  if (!is_finite(scale)) return fail(HUB_ERR_ARG, "scale must be finite");
  if (accumulate != 0 && accumulate != 1) return fail(HUB_ERR_ARG, "accumulate must be 0 or 1");
  HUB_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  const Geom g = make_geom(*lat);
  void* tmp = nullptr;
  if (!xi) {
    tmp = ctx->pool->alloc((size_t)batch * g.n * 16, stream);
    if (!tmp) return HUB_ERR_OOM;
    hipError_t e = launch_apply(g, phi, (const double2*)eta, (double2*)tmp, batch, true, stream);
    if (e != hipSuccess) {
      ctx->pool->release(tmp, stream);
      return hip_fail(e, "xi launch");
    }
    xi = (const hub_c128*)tmp;
  }
  hipError_t e = launch_force(g, phi, (const double2*)eta, (const double2*)xi, scale, accumulate, dSdphi, batch,
                              stream);
  if (tmp) ctx->pool->release(tmp, stream);
  if (e != hipSuccess) return hip_fail(e, "force launch");
  return HUB_OK;
}

hub_status hub_action(hub_ctx* ctx, const hub_lattice* lat, const hub_c128* chi, const hub_c128* eta,
                      int32_t batch, double* S, hipStream_t stream) {
  set_error("");
  if (!ctx) return fail(HUB_ERR_ARG, "ctx is NULL");
  hub_status s = check_lattice(lat);
  if (s) return s;
  if ((s = check_batch(batch))) return s;
  if (!chi || !eta || !S) return fail(HUB_ERR_ARG, "NULL buffer");
  HUB_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  const Geom g = make_geom(*lat);
  const int nt = ntiles_of(g.n);
  const size_t part_bytes = (size_t)batch * nt * sizeof(double);
  char* ws = (char*)ctx->pool->alloc(part_bytes + 64 * sizeof(double), stream);
  if (!ws) return HUB_ERR_OOM;
  double* part = (double*)ws;
  double* result = (double*)(ws + part_bytes);
  hipError_t e = launch_dot_re(g, (const double2*)chi, (const double2*)eta, batch, part, result, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(S, result, batch * sizeof(double), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  ctx->pool->release(ws, stream);
  if (e != hipSuccess) return hip_fail(e, "action");
  return HUB_OK;
}

}  // extern "C"

namespace {

hub_status check_masses(const double* mt, int32_t n) {
  if (n < 0 || n > HUB_MAX_HB_MASSES) return fail(HUB_ERR_ARG, "n must be in [0, HUB_MAX_HB_MASSES]");
  if (n > 0 && !mt) return fail(HUB_ERR_ARG, "masses is NULL");
  for (int i = 0; i < n; ++i)
    if (!is_finite(mt[i])) return fail(HUB_ERR_ARG, "masses must be finite");
  return HUB_OK;
}

// Geometry of M_{mu_i}; i = -1 is the lattice's own operator.
Geom geom_with_mass(const hub_lattice& lat, const double* mt, int i) {
  hub_lattice l = lat;
  if (i >= 0) l.ms_t = mt[i];
  return make_geom(l);
}

// Heat-bath of the n+1 pseudofermions (Sec. 5.1).  Caller holds ctx->mu, device set.
hub_status heatbath_impl(hub_ctx* ctx, const hub_lattice& lat, const double* phi, const double* mt, int n,
                         const double2* rho, double2* chi, const hub_solve_opts& o, hub_solve_info* info,
                         hipStream_t stream) {
  const size_t N = (size_t)make_geom(lat).n;
  // chi_n = M_{n-1} rho_n
  HUB_HIP(launch_apply(geom_with_mass(lat, mt, n - 1), phi, rho + n * N, chi + n * N, 1, false, stream), "apply");
  if (n == 0) return HUB_OK;
  // chi_i = M_i^{-1} M_{i-1} rho_i = M_i^dag (M_i M_i^dag)^{-1} M_{i-1} rho_i, i < n
  double2* w = (double2*)ctx->pool->alloc(2 * (size_t)n * N * 16, stream);
  if (!w) return fail(HUB_ERR_OOM, "heat-bath workspace");
  double2* y = w + (size_t)n * N;
  std::vector<System> sys((size_t)n);
  hipError_t e = hipSuccess;
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    e = launch_apply(geom_with_mass(lat, mt, i - 1), phi, rho + i * N, w + i * N, 1, false, stream);
    sys[i].g = geom_with_mass(lat, mt, i);
    sys[i].mu2 = 0.0;
    sys[i].b = w + i * N;
    sys[i].x = y + i * N;
  }
  hub_solve_opts oz = o;
  oz.use_x0 = 0;
  hub_status result = e == hipSuccess ? run_solves(ctx, sys, phi, oz, stream) : hip_fail(e, "apply");
  if (result == HUB_OK || result == HUB_ERR_NOCONV) {
    for (int i = 0; i < n && e == hipSuccess; ++i)
      e = launch_apply(sys[i].g, phi, y + i * N, chi + i * N, 1, true, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) result = hip_fail(e, "apply");
    if (info)
      for (int i = 0; i < n; ++i) info[i] = sys[i].info;
  }
  ctx->pool->release(w, stream);
  return result;
}

// Actions and force of the selected terms (Sec. 5.1, eq. (f_chi_i)); term terms[k]
// enters dSdphi with scales[k].  S and info are indexed by term.  Caller holds
// ctx->mu, device set.  Synchronises the stream.
hub_status eval_impl(hub_ctx* ctx, const hub_lattice& lat, const double* phi, const double* mt, int n,
                     const double2* chi, const std::vector<int>& terms, const std::vector<double>& scales,
                     int accumulate, double* dSdphi, double* S, double2* eta, const hub_solve_opts& o,
                     hub_solve_info* info, hipStream_t stream) {
  const Geom g = make_geom(lat);
  const size_t N = (size_t)g.n;
  const int T = (int)terms.size();
  const int nt = ntiles_of(g.n);
  // workspace: M_i chi_i for the ratio terms, xi per term, dot partials and results
  const size_t vec_bytes = (size_t)T * N * 16;
  const size_t part_bytes = (size_t)T * nt * sizeof(double);
  char* ws = (char*)ctx->pool->alloc(2 * vec_bytes + part_bytes + 64 * sizeof(double), stream);
  if (!ws) return fail(HUB_ERR_OOM, "Hasenbusch workspace");
  double2* wv = (double2*)ws;
  double2* xv = (double2*)(ws + vec_bytes);
  double* part = (double*)(ws + 2 * vec_bytes);
  double* res = (double*)(ws + 2 * vec_bytes + part_bytes);
  std::vector<System> sys((size_t)T);
  std::vector<const double2*> rhs((size_t)T);
  hipError_t e = hipSuccess;
  for (int k = 0; k < T && e == hipSuccess; ++k) {
    const int i = terms[k];
    const int den = i == n ? n - 1 : i - 1;
    if (i == n) {
      rhs[k] = chi + i * N;
    } else {
      e = launch_apply(geom_with_mass(lat, mt, i), phi, chi + i * N, wv + k * N, 1, false, stream);
      rhs[k] = wv + k * N;
    }
    sys[k].g = geom_with_mass(lat, mt, den);
    sys[k].mu2 = 0.0;
    sys[k].b = rhs[k];
    sys[k].x = eta + i * N;
  }
  hub_status result = e == hipSuccess ? run_solves(ctx, sys, phi, o, stream) : hip_fail(e, "apply");
  if (result == HUB_OK || result == HUB_ERR_NOCONV) {
    double Sh[kMaxSys] = {0};
    for (int k = 0; k < T && e == hipSuccess; ++k) {
      const int i = terms[k];
      // S_i = Re rhs_i^dag eta_i; xi_i = M_den^dag eta_i; dS_i/dphi with xi_i (- chi_i)
      e = launch_dot_re(g, rhs[k], eta + i * N, 1, part + (size_t)k * nt, res + k, stream);
      if (e == hipSuccess) e = launch_apply(sys[k].g, phi, eta + i * N, xv + k * N, 1, true, stream);
      if (e == hipSuccess && dSdphi)
        e = launch_force(g, phi, eta + i * N, xv + k * N, scales[k], (k == 0) ? accumulate : 1, dSdphi, 1,
                         stream, i == n ? nullptr : chi + i * N);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(Sh, res, T * sizeof(double), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      result = hip_fail(e, "Hasenbusch force");
    } else {
      for (int k = 0; k < T; ++k) {
        if (S) S[terms[k]] = Sh[k];
        if (info) info[terms[k]] = sys[k].info;
      }
    }
  }
  ctx->pool->release(ws, stream);
  return result;
}

}  // namespace

extern "C" {

hub_status hub_hasenbusch_heatbath(hub_ctx* ctx, const hub_lattice* lat, const double* phi, const double* mt,
                                   int32_t n, const hub_c128* rho, hub_c128* chi, const hub_solve_opts* opts,
                                   hub_solve_info* info, hipStream_t stream) {
  set_error("");
  if (!ctx) return fail(HUB_ERR_ARG, "ctx is NULL");
  hub_status s = check_lattice(lat);
  if (s) return s;
  if ((s = check_masses(mt, n))) return s;
  if (!phi || !rho || !chi || (n > 0 && !info)) return fail(HUB_ERR_ARG, "NULL buffer");
  if ((const void*)rho == (const void*)chi) return fail(HUB_ERR_ARG, "rho and chi must not overlap");
  hub_solve_opts o;
  hub_default_opts(&o);
  if (opts) o = *opts;
  o.use_x0 = 0;
  if ((s = check_opts(o))) return s;
  std::lock_guard<std::mutex> lk(ctx->mu);
  HUB_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  s = heatbath_impl(ctx, *lat, phi, mt, n, (const double2*)rho, (double2*)chi, o, info, stream);
  if (s == HUB_OK && n == 0) HUB_HIP(hipStreamSynchronize(stream), "heat-bath");
  return s;
}

hub_status hub_hasenbusch_force(hub_ctx* ctx, const hub_lattice* lat, const double* phi, const double* mt,
                                int32_t n, const hub_c128* chi, uint32_t term_mask, double scale,
                                int32_t accumulate, double* dSdphi, double* S, hub_c128* eta,
                                const hub_solve_opts* opts, hub_solve_info* info, hipStream_t stream) {
  set_error("");
  if (!ctx) return fail(HUB_ERR_ARG, "ctx is NULL");
  hub_status s = check_lattice(lat);
  if (s) return s;
  if ((s = check_masses(mt, n))) return s;
  if (!phi || !chi || !dSdphi || !eta || !info) return fail(HUB_ERR_ARG, "NULL buffer");
  if ((const void*)chi == (const void*)eta) return fail(HUB_ERR_ARG, "chi and eta must not overlap");
  if (term_mask == 0 || (n < 31 && (term_mask >> (n + 1)) != 0))
    return fail(HUB_ERR_ARG, "term_mask must select terms in [0, n]");
  if (!is_finite(scale)) return fail(HUB_ERR_ARG, "scale must be finite");
  if (accumulate != 0 && accumulate != 1) return fail(HUB_ERR_ARG, "accumulate must be 0 or 1");
  hub_solve_opts o;
  hub_default_opts(&o);
  if (opts) o = *opts;
  if ((s = check_opts(o))) return s;
  std::lock_guard<std::mutex> lk(ctx->mu);
  HUB_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  std::vector<int> terms;
  for (int i = 0; i <= n; ++i)
    if (term_mask & (1u << i)) terms.push_back(i);
  const std::vector<double> scales(terms.size(), scale);
  return eval_impl(ctx, *lat, phi, mt, n, (const double2*)chi, terms, scales, accumulate, dSdphi, S,
                   (double2*)eta, o, info, stream);
}

}  // extern "C"

namespace {

hub_status check_hmc(const hub_hmc_params* p, MdSchedule* sched) {
  if (!p) return fail(HUB_ERR_ARG, "params is NULL");
  hub_status s = check_masses(p->mt, p->n);
  if (s) return s;
  if (!is_finite(p->U_t) || p->U_t <= 0.0) return fail(HUB_ERR_ARG, "U_t must be finite and > 0");
  if ((p->flags & ~HUB_HMC_CHI_GIVEN) != 0) return fail(HUB_ERR_ARG, "unknown hub_hmc_params.flags");
  if ((long long)p->n_md * (p->n + 1) > (1LL << 22)) return fail(HUB_ERR_ARG, "n_md too large");
  std::string err;
  if (!sched->build(p->n, p->n_scale, p->n_md, p->traj_length, p->zeta, &err)) return fail(HUB_ERR_ARG, err);
  return HUB_OK;
}

}  // namespace

extern "C" {

hub_status hub_md_schedule(const hub_hmc_params* params, hub_md_op* ops, int32_t max_ops, int32_t* count) {
  set_error("");
  if (!count) return fail(HUB_ERR_ARG, "count is NULL");
  MdSchedule sched;
  hub_status s = check_hmc(params, &sched);
  if (s) return s;
  *count = (int32_t)sched.ops.size();
  if (ops) {
    if (max_ops < (int32_t)sched.ops.size()) return fail(HUB_ERR_ARG, "max_ops smaller than the schedule");
    for (size_t k = 0; k < sched.ops.size(); ++k) {
      std::memset(&ops[k], 0, sizeof(hub_md_op));
      ops[k].kind = sched.ops[k].kind;
      ops[k].eps = sched.ops[k].eps;
      for (int l = 0; l <= params->n; ++l) ops[k].coef[l] = sched.ops[k].coef[l];
    }
  }
  return HUB_OK;
}

hub_status hub_hmc_trajectory(hub_ctx* ctx, const hub_lattice* lat, double* phi, double* pi, const hub_c128* rho,
                              double u, const hub_hmc_params* params, const hub_solve_opts* opts,
                              hub_hmc_info* info, hipStream_t stream) {
  set_error("");
  if (!ctx) return fail(HUB_ERR_ARG, "ctx is NULL");
  hub_status s = check_lattice(lat);
  if (s) return s;
  MdSchedule sched;
  if ((s = check_hmc(params, &sched))) return s;
  if (!phi || !pi || !rho || !info) return fail(HUB_ERR_ARG, "NULL buffer");
  if (!is_finite(u) || u < 0.0 || u > 1.0) return fail(HUB_ERR_ARG, "u must be in [0, 1]");
  hub_solve_opts o;
  hub_default_opts(&o);
  if (opts) o = *opts;
  if ((s = check_opts(o))) return s;
  std::lock_guard<std::mutex> lk(ctx->mu);
  HUB_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  std::memset(info, 0, sizeof(*info));
  const int n = params->n;
  const double* mt = params->mt;
  const Geom g = make_geom(*lat);
  const size_t N = (size_t)g.n;
  const int nt2 = ntiles_of(g.n / 2);
  // workspace: phi at the start (for a rejection), chi and eta per term, the summed
  // pseudofermion force G, dot partials and results
  const size_t fld = N * sizeof(double), vec = (size_t)(n + 1) * N * 16;
  const size_t part_bytes = 2 * (size_t)nt2 * sizeof(double);
  char* ws = (char*)ctx->pool->alloc(2 * fld + 2 * vec + part_bytes + 64 * sizeof(double), stream);
  if (!ws) return fail(HUB_ERR_OOM, "HMC workspace");
  double* phi0 = (double*)ws;
  double* G = (double*)(ws + fld);
  double2* chi = (double2*)(ws + 2 * fld);
  double2* eta = (double2*)(ws + 2 * fld + vec);
  double* part = (double*)(ws + 2 * fld + 2 * vec);
  double* res = (double*)(ws + 2 * fld + 2 * vec + part_bytes);
  hub_status result = HUB_OK;
  auto hip_check = [&](hipError_t e, const char* where) {
    if (e != hipSuccess && result == HUB_OK) result = hip_fail(e, where);
    return result == HUB_OK;
  };
  // phi^2 / (2 U~) and pi^2 / 2 through the complex dot kernel on (re, im) pairs (N is even)
  Geom gh = g;
  gh.n = g.n / 2;
  auto quadratic = [&](double* gauge, double* kin) {
    double h[2] = {0, 0};
    if (!hip_check(launch_dot_re(gh, (const double2*)phi, (const double2*)phi, 1, part, res, stream), "norm"))
      return false;
    if (!hip_check(launch_dot_re(gh, (const double2*)pi, (const double2*)pi, 1, part + nt2, res + 1, stream),
                   "norm"))
      return false;
    if (!hip_check(hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, stream), "norm")) return false;
    if (!hip_check(hipStreamSynchronize(stream), "norm")) return false;
    *gauge = 0.5 * h[0] / params->U_t;
    *kin = 0.5 * h[1];
    return true;
  };
  std::vector<double> S(n + 1, 0.0), S0(n + 1, 0.0);
  std::vector<hub_solve_info> sinfo(n + 1);
  std::vector<int> all(n + 1);
  for (int i = 0; i <= n; ++i) all[i] = i;
  bool evaluated = false;  // every term has a solution in eta (warm starts allowed)
  auto evaluate = [&](const std::vector<int>& terms, const std::vector<double>& scales, double* dS) {
    hub_solve_opts oe = o;
    if (!evaluated) oe.use_x0 = 0;
    const hub_status st = eval_impl(ctx, *lat, phi, mt, n, chi, terms, scales, 0, dS, S.data(), eta, oe,
                                    sinfo.data(), stream);
    if (st != HUB_OK) {
      if (result == HUB_OK) result = st;
      return false;
    }
    evaluated = evaluated || terms.size() == (size_t)(n + 1);
    for (int t : terms) {
      info->force_evals[t]++;
      info->inner_iters += sinfo[t].inner_iters;
    }
    return true;
  };
  double g0 = 0, k0 = 0, g1 = 0, k1 = 0;
  bool saved = false;
  do {
    if (!hip_check(hipMemcpyAsync(phi0, phi, fld, hipMemcpyDeviceToDevice, stream), "copy")) break;
    saved = true;
    if (params->flags & HUB_HMC_CHI_GIVEN) {
      if (!hip_check(hipMemcpyAsync(chi, rho, vec, hipMemcpyDeviceToDevice, stream), "copy")) break;
    } else if ((result = heatbath_impl(ctx, *lat, phi, mt, n, (const double2*)rho, chi, o, nullptr, stream)) !=
               HUB_OK) {
      break;
    }
    if (!quadratic(&g0, &k0)) break;
    // the pseudofermion actions at the start; the first kick group's forces come from the same solves
    const MdOp& first = sched.ops.front();
    bool first_all = first.kind == 1;
    for (int i = 0; i <= n && first_all; ++i) first_all = first.coef[i] != 0.0;
    if (!first_all) {
      if (!evaluate(all, std::vector<double>(n + 1, 0.0), nullptr)) break;
      S0 = S;
    }
    bool ok = true;
    for (size_t k = 0; k < sched.ops.size() && ok; ++k) {
      const MdOp& op = sched.ops[k];
      if (op.kind == 0) {
        ok = hip_check(launch_md_drift(phi, pi, op.eps, g.n, stream), "drift");
        info->drifts++;
        continue;
      }
      std::vector<int> terms;
      std::vector<double> scales;
      for (int l = 0; l <= n; ++l)
        if (op.coef[l] != 0.0) {
          terms.push_back(l);
          scales.push_back(op.coef[l]);
        }
      ok = evaluate(terms, scales, G);
      if (!ok) break;
      if (k == 0) S0 = S;
      // pi -= sum_l coef_l dS_l/dphi - coef_n phi / U~ (the gauge force rides with level n)
      ok = hip_check(launch_md_kick(pi, phi, G, op.coef[n] / params->U_t, g.n, stream), "kick");
      info->kick_groups++;
    }
    if (!ok) break;
    // the pseudofermion actions at the end (the last kick group holds every level unless zeta = 0)
    const MdOp& last = sched.ops.back();
    bool last_all = last.kind == 1;
    for (int i = 0; i <= n && last_all; ++i) last_all = last.coef[i] != 0.0;
    if (!last_all && !evaluate(all, std::vector<double>(n + 1, 0.0), nullptr)) break;
    if (!quadratic(&g1, &k1)) break;
  } while (false);
  if (result == HUB_OK) {
    double sf0 = 0, sf1 = 0;
    for (int i = 0; i <= n; ++i) {
      sf0 += S0[i];
      sf1 += S[i];
    }
    info->H0 = g0 + k0 + sf0;
    info->H1 = g1 + k1 + sf1;
    info->dH = info->H1 - info->H0;
    info->accepted = (std::isfinite(info->dH) && u < std::exp(-info->dH)) ? 1 : 0;
    if (!info->accepted) hip_check(hipMemcpyAsync(phi, phi0, fld, hipMemcpyDeviceToDevice, stream), "restore");
    hip_check(hipStreamSynchronize(stream), "trajectory");
  } else if (saved) {
    // a failed trajectory leaves phi as it was (best effort after a device error)
    if (hipMemcpyAsync(phi, phi0, fld, hipMemcpyDeviceToDevice, stream) == hipSuccess)
      (void)hipStreamSynchronize(stream);
  }
  ctx->pool->release(ws, stream);
  return result;
}

}  // extern "C"

namespace {

// Extreme eigenvalues of the symmetric tridiagonal matrix (diagonal d, off-diagonal e)
// by Sturm-sequence bisection.
void tridiag_extremes(const std::vector<double>& d, const std::vector<double>& e, double* lo, double* hi) {
  const int k = (int)d.size();
  double gl = d[0], gu = d[0];
  for (int j = 0; j < k; ++j) {
    const double rad = (j > 0 ? std::fabs(e[j - 1]) : 0.0) + (j + 1 < k ? std::fabs(e[j]) : 0.0);
    gl = std::min(gl, d[j] - rad);
    gu = std::max(gu, d[j] + rad);
  }
  // eigenvalues below x
  auto below = [&](double x) {
    int c = 0;
    double q = 1.0;
    for (int j = 0; j < k; ++j) {
      q = (d[j] - x) - (j > 0 ? e[j - 1] * e[j - 1] / q : 0.0);
      if (q == 0.0) q = -1e-300;
      if (q < 0.0) ++c;
    }
    return c;
  };
  auto solve = [&](int target) {  // smallest x with below(x) >= target
    double a = gl, b = gu;
    for (int it = 0; it < 200 && b - a > 1e-15 * std::max(std::fabs(a), std::fabs(b)); ++it) {
      const double m = 0.5 * (a + b);
      if (below(m) >= target) b = m; else a = m;
    }
    return 0.5 * (a + b);
  };
  *lo = solve(1);
  *hi = solve(k);
}

}  // namespace

extern "C" {

hub_status hub_solve_multishift(hub_ctx* ctx, const hub_lattice* lat, const double* phi, const double* mu2,
                                int32_t nshift, const hub_c128* b, hub_c128* x, const hub_solve_opts* opts,
                                hub_solve_info* info, double* lambda, hipStream_t stream) {
  set_error("");
  if (!ctx) return fail(HUB_ERR_ARG, "ctx is NULL");
  hub_status s = check_lattice(lat);
  if (s) return s;
  if (nshift < 1 || nshift > HUB_MAX_SHIFTS) return fail(HUB_ERR_ARG, "nshift must be in [1, HUB_MAX_SHIFTS]");
  if (!phi || !mu2 || !b || !x || !info) return fail(HUB_ERR_ARG, "NULL buffer");
  for (int k = 0; k < nshift; ++k)
    if (!is_finite(mu2[k]) || mu2[k] < 0) return fail(HUB_ERR_ARG, "mu2 must be finite and >= 0");
  hub_solve_opts o;
  hub_default_opts(&o);
  if (opts) o = *opts;
  o.solver = HUB_CG_FP64;
  if ((s = check_opts(o))) return s;
  std::lock_guard<std::mutex> lk(ctx->mu);
  HUB_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  const Geom g = make_geom(*lat);
  const size_t N = (size_t)g.n;
  const int nt = ntiles_of(g.n);
  int bi = 0;
  for (int k = 1; k < nshift; ++k)
    if (mu2[k] < mu2[bi]) bi = k;
  const int ns = nshift - 1;
  const int maxit = o.max_iter;
  // workspace: r, p pair, u, the shifted directions, partials, scalars, descriptor, Lanczos history
  const size_t vecs = (size_t)(4 + ns) * N * 16;
  const size_t parts = 2 * (size_t)nt * sizeof(double);
  const size_t hist_bytes = (2 * (size_t)maxit + 2) * sizeof(double);
  const size_t tail = ((sizeof(MsScal) + 255) / 256) * 256 + ((sizeof(MsDesc) + 255) / 256) * 256;
  char* ws = (char*)ctx->pool->alloc(vecs + parts + tail + hist_bytes, stream);
  if (!ws) return fail(HUB_ERR_OOM, "multi-shift workspace");
  double2* v = (double2*)ws;
  MsDesc h;
  std::memset(&h, 0, sizeof(h));
  h.g = g;
  h.phi = phi;
  h.mu2 = mu2[bi];
  h.b = (const double2*)b;
  h.x = (double2*)x + bi * N;
  h.r = v;
  h.p[0] = v + N;
  h.p[1] = v + 2 * N;
  h.u = v + 3 * N;
  std::vector<int> order;  // shifted systems in input order (without the base)
  for (int k = 0; k < nshift; ++k)
    if (k != bi) order.push_back(k);
  for (int q = 0; q < ns; ++q) {
    h.xs[q] = (double2*)x + (size_t)order[q] * N;
    h.ps[q] = v + (size_t)(4 + q) * N;
    h.sigma[q] = mu2[order[q]] - mu2[bi];
  }
  h.ns = ns;
  h.ntiles = nt;
  h.part1 = (double*)(ws + vecs);
  h.part2 = h.part1 + nt;
  char* t = ws + vecs + parts;
  h.sc = (MsScal*)t;
  MsDesc* dd = (MsDesc*)(t + ((sizeof(MsScal) + 255) / 256) * 256);
  h.hist = (double*)(t + tail);
  h.tol2 = o.tol * o.tol;
  h.maxit = maxit;
  hub_status result = HUB_OK;
  int iters = 0;
  std::vector<double> hist;
  do {
    hipError_t e = hipMemcpyAsync(dd, &h, sizeof(h), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = launch_ms_start(dd, nt, stream);
    if (e != hipSuccess) {
      result = hip_fail(e, "multi-shift start");
      break;
    }
    int it = 0;
    for (;;) {
      for (int j = 0; j < o.check_every && e == hipSuccess; ++j) e = launch_ms_iter(dd, nt, it++, stream);
      int flags[2] = {0, 0};  // active, iters
      if (e == hipSuccess) e = hipMemcpyAsync(flags, &h.sc->active, sizeof(int), hipMemcpyDeviceToHost, stream);
      if (e == hipSuccess) e = hipMemcpyAsync(flags + 1, &h.sc->iters, sizeof(int), hipMemcpyDeviceToHost, stream);
      if (e == hipSuccess) e = hipStreamSynchronize(stream);
      if (e != hipSuccess) break;
      if (!flags[0]) {
        iters = flags[1];
        break;
      }
      if (it > maxit + o.check_every) {  // unreachable: the kernels stop at maxit
        iters = maxit;
        break;
      }
    }
    if (e != hipSuccess) {
      result = hip_fail(e, "multi-shift iterations");
      break;
    }
    if (lambda && iters > 0) {
      hist.resize(2 * (size_t)iters);
      e = hipMemcpyAsync(hist.data(), h.hist, hist.size() * sizeof(double), hipMemcpyDeviceToHost, stream);
      if (e == hipSuccess) e = hipStreamSynchronize(stream);
      if (e != hipSuccess) {
        result = hip_fail(e, "Lanczos coefficients");
        break;
      }
    }
  } while (false);
  ctx->pool->release(ws, stream);
  if (result != HUB_OK) return result;
  // certify every shift by its FP64 true residual (a warm-started CG that stops at
  // once when the shifted iterate already meets the tolerance)
  std::vector<System> sys((size_t)nshift);
  for (int k = 0; k < nshift; ++k) {
    sys[k].g = g;
    sys[k].mu2 = mu2[k];
    sys[k].b = (const double2*)b;
    sys[k].x = (double2*)x + (size_t)k * N;
  }
  hub_solve_opts oc = o;
  oc.use_x0 = 1;
  result = run_solves(ctx, sys, phi, oc, stream);
  if (result != HUB_OK && result != HUB_ERR_NOCONV) return result;
  for (int k = 0; k < nshift; ++k) {
    info[k] = sys[k].info;
    info[k].outer_iters = iters;  // shared Krylov iterations (the polish count is in inner_iters)
  }
  if (lambda) {
    lambda[0] = lambda[1] = 0.0;
    if (iters > 0) {
      std::vector<double> dg((size_t)iters), off(iters > 1 ? (size_t)iters - 1 : 0);
      for (int j = 0; j < iters; ++j) {
        const double a = hist[2 * j];
        dg[j] = 1.0 / a + (j > 0 ? hist[2 * (j - 1) + 1] / hist[2 * (j - 1)] : 0.0);
        if (j + 1 < iters) off[j] = std::sqrt(hist[2 * j + 1]) / a;
      }
      tridiag_extremes(dg, off, &lambda[0], &lambda[1]);
      lambda[0] -= mu2[bi];
      lambda[1] -= mu2[bi];
    }
  }
  return result;
}

hub_status hub_hasenbusch_masses(double lambda_min, double lambda_max, int32_t n, double* mu) {
  set_error("");
  if (!mu) return fail(HUB_ERR_ARG, "mu is NULL");
  if (n < 1 || n > HUB_MAX_HB_MASSES) return fail(HUB_ERR_ARG, "n must be in [1, HUB_MAX_HB_MASSES]");
  if (!is_finite(lambda_min) || !is_finite(lambda_max) || !(lambda_min > 0.0) || !(lambda_max > lambda_min))
    return fail(HUB_ERR_ARG, "need 0 < lambda_min < lambda_max");
  for (int i = 0; i < n; ++i) mu[i] = lambda_min * std::pow(lambda_max / lambda_min, (double)(i + 1) / (n + 1));
  return HUB_OK;
}

hub_status hub_submit(hub_ctx* ctx, const hub_request* req, uint64_t* ticket) {
  set_error("");
  if (!ctx || !req || !ticket) return fail(HUB_ERR_ARG, "NULL argument");
  hub_status s = check_lattice(&req->lat);
  if (s) return s;
  if ((s = check_opts(req->opts))) return s;
  if (!req->phi || !req->chi || !req->x_out) return fail(HUB_ERR_ARG, "NULL buffer");
  if (!is_finite(req->mu2) || req->mu2 < 0) return fail(HUB_ERR_ARG, "mu2 must be finite and >= 0");
  Server* srv;
  {
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    if (!ctx->server) ctx->server.reset(new Server(ctx));
    srv = ctx->server.get();
  }
  return srv->submit(*req, ticket);
}

hub_status hub_poll(hub_ctx* ctx, uint64_t ticket, int32_t* done, hub_solve_info* info) {
  set_error("");
  if (!ctx || !done) return fail(HUB_ERR_ARG, "NULL argument");
  Server* srv;
  {
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    srv = ctx->server.get();
  }
  if (!srv) return fail(HUB_ERR_NOTFOUND, "unknown ticket");
  return srv->poll(ticket, done, info);
}

hub_status hub_profile_enable(hub_ctx* ctx, int32_t enable) {
  set_error("");
  if (!ctx) return fail(HUB_ERR_ARG, "ctx is NULL");
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->profiling = enable != 0;
  for (auto& kv : ctx->engines) kv.second->set_profiling(ctx->profiling);
  return HUB_OK;
}

hub_status hub_profile_read(hub_ctx* ctx, hub_kernel_stat* out, int32_t max, int32_t* count) {
  set_error("");
  if (!ctx || !out || !count) return fail(HUB_ERR_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(ctx->mu);
  static const char* names[2][2] = {{"cg1_f64", "cg2_f64"}, {"cg1_c64", "cg2_c64"}};
  int n = 0;
  for (int sp = 0; sp < 2; ++sp)
    for (int st = 0; st < 2; ++st) {
      if (n >= max) break;
      hub_kernel_stat k;
      std::memset(&k, 0, sizeof(k));
      std::strncpy(k.name, names[sp][st], sizeof(k.name) - 1);
      for (auto& kv : ctx->engines) {
        const Engine::KernelStat& e = kv.second->stat[sp][st];
        k.launches += e.launches;
        k.total_ms += e.ms;
        k.bytes += e.bytes;
      }
      out[n++] = k;
    }
  *count = n;
  return HUB_OK;
}

}  // extern "C"
