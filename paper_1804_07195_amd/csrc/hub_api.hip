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

#include "hub_api_internal.h"

using namespace hub;
using namespace hub::api;

namespace hub {
namespace api {

// Device scratch of hub_apply_normal_noalloc.  In host code this name stands for the
// symbol, not a device address: kernels get the address that hipGetSymbolAddress
// returns on each device, recorded once per device at hub_create.
static __device__ __align__(256) unsigned char scratch[HUB_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static void* g_scratch[kMaxDevices] = {nullptr};
static std::mutex g_scratch_mu;

// The scratch address on `device` (the current device), looked up once.
static hipError_t scratch_on(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[device] = p;
  }
  *out = g_scratch[device];
  return hipSuccess;
}

hub_status fail(hub_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

hub_status hip_fail(hipError_t e, const char* where) {
  return fail(HUB_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}


bool is_finite(double v) { return std::isfinite(v); }

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b || na == 0 || nb == 0) return false;
  const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
  return pa < pb + nb && pb < pa + na;
}

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

// One served request.
struct Ticket {
  hub_request req;
  System sys;
  std::atomic<int> state{0};  // 0 queued, 1 running, 2 done
  hub_solve_info info{};
  hub_status status = HUB_OK;  // final status, reported by hub_poll once done
};


}  // namespace api
}  // namespace hub


namespace hub {
namespace api {

// Continuous batching: admits queued requests whenever an engine slot and their
// workspace fit, and advances all admitted requests together.
class Server {
 public:
  explicit Server(hub_ctx* ctx) : ctx_(ctx) {
    if (hipSetDevice(ctx->device) != hipSuccess || hipStreamCreateWithFlags(&st_, hipStreamNonBlocking) != hipSuccess) {
      st_ = nullptr;
      return;
    }
    engine_.reset(new Engine(ctx->pool.get(), st_));
    if (!engine_->ok()) return;
    thread_ = std::thread([this] { run(); });
  }
  // False if the stream, the engine or the thread could not be set up.
  bool ok() const { return thread_.joinable(); }
  ~Server() {
    if (thread_.joinable()) {
      {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
      }
      cv_.notify_all();
      thread_.join();
    }
    engine_.reset();
    if (st_) (void)hipStreamDestroy(st_);
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
    const hub_status st = it->second->status;
    tickets_.erase(it);
    if (st == HUB_ERR_NOCONV) set_error("iteration limit reached before the tolerance");
    if (st == HUB_ERR_ARG) set_error("non-finite value in phi, chi or the initial guess");
    if (st == HUB_ERR_HIP) set_error("a HIP runtime call failed while the request ran");
    return st;
  }

 private:
  void run() {
    (void)hipSetDevice(ctx_->device);  // set successfully by the constructor on this device
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
        const Engine::AddResult ar = engine_->add(&s);
        if (ar == Engine::ADD_NO_ROOM) {
          back.push_back(id);  // retried once running requests release workspace or slots
          continue;
        }
        if (ar != Engine::ADD_OK) {
          // a HIP failure while joining: the request ends with that status
          t->status = HUB_ERR_HIP;
          t->info = hub_solve_info{};
          t->state = 2;
          continue;
        }
        t->state = 1;
        running_.push_back(t);
      }
      if (!back.empty()) {
        std::lock_guard<std::mutex> lk(mu_);
        for (auto it = back.rbegin(); it != back.rend(); ++it) queue_.push_front(*it);
      }
      if (engine_->count() == 0) {
        // nothing runs: a request that did not fit waits for workspace held elsewhere
        if (!back.empty()) std::this_thread::sleep_for(std::chrono::milliseconds(1));
        continue;
      }
      if (engine_->step() != hipSuccess) {
        // a HIP failure: fail every running request
        for (auto& t : running_) {
          t->sys.status = HUB_ERR_HIP;
          t->status = HUB_ERR_HIP;
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
    hub_status st = s->status;
    if (st == HUB_OK || st == HUB_ERR_NOCONV) {
      // S and the force from the (last) iterate
      if (engine_->finalize(s, (const double2*)r.chi, r.dSdphi_out, &S) != hipSuccess) {
        s->info.converged = 0;
        st = HUB_ERR_HIP;
      }
    }
    if (r.S_out) *r.S_out = S;
    t->status = st;
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
  std::unique_ptr<Engine> e(new Engine(ctx->pool.get(), st));
  if (!e->ok()) {
    set_error("could not allocate the solver engine's buffers");
    return nullptr;
  }
  e->set_profiling(ctx->profiling);
  Engine* p = e.get();
  ctx->engines[st] = std::move(e);
  return p;
}

}  // namespace api
}  // namespace hub

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
  o->check_every = 8;
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
  void* scr = nullptr;
  HUB_HIP(scratch_on(device, &scr), "hipGetSymbolAddress(scratch)");
  hub_ctx* c = new hub_ctx;
  c->device = device;
  c->scratch = scr;
  c->pool.reset(new Pool(device, hbm_budget_bytes ? hbm_budget_bytes : freeb / 4 * 3));
  *ctx = c;
  return HUB_OK;
}

hub_status hub_destroy(hub_ctx* ctx) {
  if (!ctx) return fail(HUB_ERR_ARG, "ctx is NULL");
  (void)hipSetDevice(ctx->device);
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
  const Geom g = make_geom(*lat);
  const size_t vb = (size_t)batch * g.n * sizeof(hub_c128);
  if (overlaps(x, vb, y, vb) || overlaps(phi, (size_t)g.n * 8, y, vb))
    return fail(HUB_ERR_ARG, "y must not overlap x or phi");
  HUB_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  HUB_HIP(launch_apply(g, phi, (const double2*)x, (double2*)y, batch, dag, st, true), "apply launch");
  return HUB_OK;
}

hub_status hub_apply_fields(hub_ctx* ctx, const hub_lattice* lat, const double* phi, int32_t per_field, int32_t dag,
                            const hub_c128* x, hub_c128* y, int32_t batch, hipStream_t stream) {
  set_error("");
  if (!ctx) return fail(HUB_ERR_ARG, "ctx is NULL");
  hub_status s = check_lattice(lat);
  if (s) return s;
  if ((s = check_batch(batch))) return s;
  if (per_field < 1 || batch % per_field != 0) return fail(HUB_ERR_ARG, "batch must be a multiple of per_field");
  if (dag != 0 && dag != 1) return fail(HUB_ERR_ARG, "dag must be 0 or 1");
  if (!phi || !x || !y) return fail(HUB_ERR_ARG, "NULL buffer");
  const Geom g = make_geom(*lat);
  const int nfield = batch / per_field;
  const size_t vb = (size_t)batch * g.n * sizeof(hub_c128);
  if (overlaps(x, vb, y, vb) || overlaps(phi, (size_t)nfield * g.n * 8, y, vb))
    return fail(HUB_ERR_ARG, "y must not overlap x or phi");
  HUB_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  for (int f = 0; f < nfield; ++f) {
    const size_t off = (size_t)f * per_field * g.n;
    HUB_HIP(launch_apply(g, phi + (size_t)f * g.n, (const double2*)(x + off), (double2*)(y + off), per_field,
                         dag != 0, stream, true),
            "apply launch");
  }
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
  {
    const Geom gg = make_geom(*lat);
    const size_t vb = (size_t)batch * gg.n * sizeof(hub_c128);
    if (overlaps(x, vb, y, vb) || overlaps(phi, (size_t)gg.n * 8, y, vb))
      return fail(HUB_ERR_ARG, "y must not overlap x or phi");
  }
  double m2[kMaxSys] = {0};
  for (int b = 0; b < batch; ++b) {
    if (!is_finite(mu2[b]) || mu2[b] < 0) return fail(HUB_ERR_ARG, "mu2 must be finite and >= 0");
    m2[b] = mu2[b];
  }
  HUB_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  const Geom g = make_geom(*lat);
  // two passes, u = M^dagger x then y = M u + mu2 x: faster here than the one-pass
  // 12-point form, whose extra neighbour loads cost more than the bytes it saves
  double2* u = (double2*)ctx->pool->alloc((size_t)batch * g.n * 16, stream);
  if (!u) return fail(HUB_ERR_OOM, "workspace for M^dagger x");
  hipError_t e = launch_apply(g, phi, (const double2*)x, u, batch, true, stream);
  if (e == hipSuccess) e = launch_normal2(g, phi, m2, u, (const double2*)x, (double2*)y, batch, stream);
  ctx->pool->release(u, stream);
  if (e != hipSuccess) return hip_fail(e, "normal operator launch");
  return HUB_OK;
}

hub_status hub_apply_normal_noalloc(hub_ctx* ctx, const hub_lattice* lat, const double* phi, const double* mu2,
                                    const hub_c128* x, hub_c128* y, int32_t batch, hipStream_t stream) {
  set_error("");
  if (!ctx) return fail(HUB_ERR_ARG, "ctx is NULL");
  hub_status s = check_lattice(lat);
  if (s) return s;
  if ((s = check_batch(batch))) return s;
  if (!phi || !x || !y || !mu2) return fail(HUB_ERR_ARG, "NULL buffer");
  const Geom g = make_geom(*lat);
  const size_t vb = (size_t)batch * g.n * sizeof(hub_c128);
  if (vb > HUB_NOALLOC_SCRATCH_BYTES)
    return fail(HUB_ERR_ARG, "batch * N * 16 bytes exceed HUB_NOALLOC_SCRATCH_BYTES (" +
                                 std::to_string(vb) + " > " + std::to_string((size_t)HUB_NOALLOC_SCRATCH_BYTES) + ")");
  if (overlaps(x, vb, y, vb) || overlaps(phi, (size_t)g.n * 8, y, vb)) return fail(HUB_ERR_ARG, "y must not overlap x or phi");
  double m2[kMaxSys] = {0};
  for (int b = 0; b < batch; ++b) {
    if (!is_finite(mu2[b]) || mu2[b] < 0) return fail(HUB_ERR_ARG, "mu2 must be finite and >= 0");
    m2[b] = mu2[b];
  }
  if (!ctx->scratch) return fail(HUB_ERR_HIP, "no scratch address for this device");
  HUB_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  // u = M^dagger x into the scratch (every entry written before it is read), then
  // y = M u + mu2 x: the kernels of hub_apply_normal
  double2* u = (double2*)ctx->scratch;
  hipError_t e = launch_apply(g, phi, (const double2*)x, u, batch, true, stream);
  if (e == hipSuccess) e = launch_normal2(g, phi, m2, u, (const double2*)x, (double2*)y, batch, stream);
  if (e != hipSuccess) return hip_fail(e, "normal operator launch");
  return HUB_OK;
}

}  // extern "C"

namespace hub {
namespace api {

hub_status run_solves(hub_ctx* ctx, std::vector<System>& sys, const hub_solve_opts& o, hipStream_t stream) {
  Engine* eng = engine_for(ctx, stream);
  if (!eng) return HUB_ERR_OOM;
  // the phase e^{i phi} once per distinct phi (complex64 too for the mixed solver, and the
  // (cos, sin) table of the single-workgroup CG for small systems)
  const bool want32 = o.solver == HUB_FGMRES_MIXED;
  struct Phase {
    double2* p64;
    float* p32;
    float2* cs32;
  };
  std::map<const double*, Phase> phase;
  std::vector<void*> owned;
  hub_status result = HUB_OK;
  for (System& sy : sys) {
    if (phase.count(sy.phi)) continue;
    const bool wantcs = want32 && wg_of(sy.g.n);
    double2* p64 = (double2*)ctx->pool->alloc((size_t)sy.g.n * 16, stream);
    float* p32 = want32 ? (float*)ctx->pool->alloc((size_t)sy.g.n * 4, stream) : nullptr;
    float2* pcs = wantcs ? (float2*)ctx->pool->alloc((size_t)sy.g.n * 8, stream) : nullptr;
    if (p64) owned.push_back(p64);
    if (p32) owned.push_back(p32);
    if (pcs) owned.push_back(pcs);
    if (!p64 || (want32 && !p32) || (wantcs && !pcs)) {
      result = fail(HUB_ERR_OOM, "workspace for the phase of phi");
      break;
    }
    phase[sy.phi] = {p64, p32, pcs};
    const hipError_t e = launch_phase(sy.phi, p64, p32, sy.g.n, stream, pcs);
    if (e != hipSuccess) {
      result = hip_fail(e, "phase");
      break;
    }
  }
  size_t added = 0;
  for (System& sy : sys) {
    if (result != HUB_OK) break;
    sy.ph64 = phase[sy.phi].p64;
    sy.ph32 = phase[sy.phi].p32;
    sy.cs32 = phase[sy.phi].cs32;
    sy.opts = o;
    const Engine::AddResult ar = eng->add(&sy);
    if (ar != Engine::ADD_OK) {
      result = ar == Engine::ADD_HIP ? fail(HUB_ERR_HIP, get_error()) : fail(HUB_ERR_OOM, "solver workspace");
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
  ctx->pool->release_all(owned, stream);
  hipError_t e = hipStreamSynchronize(stream);
  if (result != HUB_OK) return result;
  if (e != hipSuccess) return hip_fail(e, "solve");
  // the first failure in this order of severity: non-finite input, then non-convergence
  for (const System& sy : sys)
    if (sy.status == HUB_ERR_ARG) result = HUB_ERR_ARG;
  for (const System& sy : sys)
    if (sy.status != HUB_OK && result == HUB_OK) result = sy.status;
  if (result == HUB_ERR_ARG) set_error("non-finite value in phi, the right-hand side or the initial guess");
  if (result == HUB_ERR_NOCONV) set_error("iteration limit reached before the tolerance");
  return result;
}

}  // namespace api
}  // namespace hub

extern "C" {

hub_status hub_solve(hub_ctx* ctx, const hub_lattice* lat, const double* phi, const double* mu2, int32_t batch,
                     const hub_c128* b, hub_c128* x, const hub_solve_opts* opts, hub_solve_info* info,
                     hipStream_t stream) {
  return hub_solve_fields(ctx, lat, phi, batch, mu2, batch, b, x, opts, info, stream);
}

hub_status hub_solve_fields(hub_ctx* ctx, const hub_lattice* lat, const double* phi, int32_t per_field,
                            const double* mu2, int32_t batch, const hub_c128* b, hub_c128* x,
                            const hub_solve_opts* opts, hub_solve_info* info, hipStream_t stream) {
  set_error("");
  if (!ctx) return fail(HUB_ERR_ARG, "ctx is NULL");
  hub_status s = check_lattice(lat);
  if (s) return s;
  if ((s = check_batch(batch))) return s;
  if (per_field < 1 || batch % per_field != 0) return fail(HUB_ERR_ARG, "batch must be a multiple of per_field");
  if (!phi || !b || !x || !mu2 || !info) return fail(HUB_ERR_ARG, "NULL buffer");
  hub_solve_opts o;
  hub_default_opts(&o);
  if (opts) o = *opts;
  if ((s = check_opts(o))) return s;
  for (int k = 0; k < batch; ++k)
    if (!is_finite(mu2[k]) || mu2[k] < 0) return fail(HUB_ERR_ARG, "mu2 must be finite and >= 0");
  const Geom g = make_geom(*lat);
  const int nfield = batch / per_field;
  {
    const size_t vb = (size_t)batch * g.n * sizeof(hub_c128);
    if (overlaps(b, vb, x, vb) || overlaps(phi, (size_t)nfield * g.n * 8, x, vb))
      return fail(HUB_ERR_ARG, "x must not overlap b or phi");
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  HUB_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  std::vector<System> sys((size_t)batch);
  for (int k = 0; k < batch; ++k) {
    sys[k].g = g;
    sys[k].mu2 = mu2[k];
    sys[k].phi = phi + (size_t)(k / per_field) * g.n;
    sys[k].b = (const double2*)(b + (size_t)k * g.n);
    sys[k].x = (double2*)(x + (size_t)k * g.n);
  }
  const hub_status result = run_solves(ctx, sys, o, stream);
  if (result != HUB_OK && result != HUB_ERR_NOCONV && result != HUB_ERR_ARG) return result;
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
  const Geom g = make_geom(*lat);
  {
    const size_t vb = (size_t)batch * g.n * sizeof(hub_c128), fb = (size_t)batch * g.n * 8;
    if (overlaps(dSdphi, fb, eta, vb) || overlaps(dSdphi, fb, xi, vb) || overlaps(dSdphi, fb, phi, (size_t)g.n * 8))
      return fail(HUB_ERR_ARG, "dSdphi must not overlap phi, eta or xi");
  }
  HUB_HIP(hipSetDevice(ctx->device), "hipSetDevice");
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

hub_status hub_force_sum(hub_ctx* ctx, const hub_lattice* lat, const double* phi, const hub_c128* eta,
                         const hub_c128* xi, const double* scale, int32_t accumulate, double* dSdphi, int32_t batch,
                         hipStream_t stream) {
  set_error("");
  if (!ctx) return fail(HUB_ERR_ARG, "ctx is NULL");
  hub_status s = check_lattice(lat);
  if (s) return s;
  if ((s = check_batch(batch))) return s;
  if (!phi || !eta || !dSdphi || !scale) return fail(HUB_ERR_ARG, "NULL buffer");
  for (int b = 0; b < batch; ++b)
    if (!is_finite(scale[b])) return fail(HUB_ERR_ARG, "scale must be finite");
  if (accumulate != 0 && accumulate != 1) return fail(HUB_ERR_ARG, "accumulate must be 0 or 1");
  const Geom g = make_geom(*lat);
  {
    const size_t vb = (size_t)batch * g.n * sizeof(hub_c128), fb = (size_t)g.n * 8;
    if (overlaps(dSdphi, fb, eta, vb) || overlaps(dSdphi, fb, xi, vb) || overlaps(dSdphi, fb, phi, fb))
      return fail(HUB_ERR_ARG, "dSdphi must not overlap phi, eta or xi");
  }
  HUB_HIP(hipSetDevice(ctx->device), "hipSetDevice");
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
  hipError_t e = launch_force_sum(g, phi, (const double2*)eta, (const double2*)xi, scale, accumulate, dSdphi, batch,
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

extern "C" {

hub_status hub_submit(hub_ctx* ctx, const hub_request* req, uint64_t* ticket) {
  set_error("");
  if (!ctx || !req || !ticket) return fail(HUB_ERR_ARG, "NULL argument");
  hub_status s = check_lattice(&req->lat);
  if (s) return s;
  if ((s = check_opts(req->opts))) return s;
  if (!req->phi || !req->chi || !req->x_out) return fail(HUB_ERR_ARG, "NULL buffer");
  if (!is_finite(req->mu2) || req->mu2 < 0) return fail(HUB_ERR_ARG, "mu2 must be finite and >= 0");
  {
    const size_t n = 2 * (size_t)req->lat.L1 * req->lat.L2 * req->lat.Nt;
    const size_t vb = n * sizeof(hub_c128);
    if (overlaps(req->chi, vb, req->x_out, vb) || overlaps(req->phi, n * 8, req->x_out, vb))
      return fail(HUB_ERR_ARG, "x_out must not overlap chi or phi");
    if (overlaps(req->dSdphi_out, n * 8, req->x_out, vb) || overlaps(req->dSdphi_out, n * 8, req->chi, vb) ||
        overlaps(req->dSdphi_out, n * 8, req->phi, n * 8))
      return fail(HUB_ERR_ARG, "dSdphi_out must not overlap x_out, chi or phi");
  }
  Server* srv;
  {
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    if (!ctx->server) {
      std::unique_ptr<Server> sv(new Server(ctx));
      if (!sv->ok()) return fail(HUB_ERR_HIP, "could not start the serving stream and engine");
      ctx->server = std::move(sv);
    }
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

hub_status hub_profile_stream(hub_ctx* ctx, const double* phi, const hub_c128* x, hub_c128* y, int64_t n,
                              int32_t mode, hipStream_t stream) {
  set_error("");
  if (!ctx) return fail(HUB_ERR_ARG, "ctx is NULL");
  if (!phi || !x || !y) return fail(HUB_ERR_ARG, "NULL buffer");
  if (n < 1 || n > (1LL << 30)) return fail(HUB_ERR_ARG, "n must be in [1, 2^30]");
  if (mode < 0 || mode > 2) return fail(HUB_ERR_ARG, "mode must be 0, 1 or 2");
  const size_t vb = (size_t)n * sizeof(hub_c128);
  if (overlaps(x, vb, y, vb) || overlaps(phi, (size_t)n * 8, y, vb))
    return fail(HUB_ERR_ARG, "y must not overlap x or phi");
  HUB_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  HUB_HIP(launch_stream_bytes(phi, (const double2*)x, (double2*)y, (int)n, mode, stream), "stream launch");
  return HUB_OK;
}

hub_status hub_profile_read(hub_ctx* ctx, hub_kernel_stat* out, int32_t max, int32_t* count) {
  set_error("");
  if (!ctx || !out || !count) return fail(HUB_ERR_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(ctx->mu);
  static const char* names[2][3] = {{"cg1_f64", "cg2_f64", "cgwg_f64"}, {"cg1_c64", "cg2_c64", "cgwg_c64"}};
  int n = 0;
  for (int sp = 0; sp < 2; ++sp)
    for (int st = 0; st < 3; ++st) {
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
