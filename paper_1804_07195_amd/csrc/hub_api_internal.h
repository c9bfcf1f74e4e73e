// Internals shared by the sources of the C ABI: the context behind hub_ctx,
// argument checks, error reporting and the batched solve driver.
#pragma once

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "hub.h"
#include "hub_engine.h"

namespace hub {
namespace api {
class Server;
}  // namespace api
}  // namespace hub

struct hub_ctx {
  int device = 0;
  void* scratch = nullptr;  // device address of the no-allocation scratch on this device
  std::unique_ptr<hub::Pool> pool;
  std::mutex mu;  // serialises the synchronous calls
  std::map<hipStream_t, std::unique_ptr<hub::Engine>> engines;
  std::unique_ptr<hub::api::Server> server;
  std::mutex server_mu;
  bool profiling = false;
};

namespace hub {
namespace api {

hub_status fail(hub_status st, const std::string& msg);
hub_status hip_fail(hipError_t e, const char* where);
bool is_finite(double v);
hub_status check_lattice(const hub_lattice* lat);
hub_status check_batch(int32_t batch);
hub_status check_opts(const hub_solve_opts& o);
// True if the byte ranges [a, a + na) and [b, b + nb) intersect (device buffers of
// one allocation space; empty ranges never intersect).
bool overlaps(const void* a, size_t na, const void* b, size_t nb);
// The engine that runs the synchronous solves enqueued on stream st.
Engine* engine_for(hub_ctx* ctx, hipStream_t st);
// Solves the prepared systems (each with its own geometry, phi, shift, right-hand
// side and solution buffer) on the stream's engine, then synchronises the stream.
// The caller holds ctx->mu and has set the device.  Per-system results are in
// sys[k].info and sys[k].status; the return value is the first failure
// (HUB_ERR_NOCONV if a system stopped at its iteration limit).
hub_status run_solves(hub_ctx* ctx, std::vector<System>& sys, const hub_solve_opts& o, hipStream_t stream);

}  // namespace api
}  // namespace hub

#define HUB_HIP(expr, where)                       \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)
