// Several shifts of one right-hand side from a shared Krylov space
// (hub_solve_multishift), with the Lanczos extremes of the CG coefficients, and the
// Hasenbusch masses of eq. (mu_i_eqn) (hub_hasenbusch_masses).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "hub_api_internal.h"

using namespace hub;
using namespace hub::api;

static_assert(HUB_MAX_SHIFTS == kMsMax + 1, "multi-shift systems");

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
  {
    const size_t nn = 2 * (size_t)lat->L1 * lat->L2 * lat->Nt, vb = nn * sizeof(hub_c128);
    if (overlaps(b, vb, x, (size_t)nshift * vb) || overlaps(phi, nn * 8, x, (size_t)nshift * vb))
      return fail(HUB_ERR_ARG, "x must not overlap b or phi");
  }
  hub_solve_opts o;
  hub_default_opts(&o);
  if (opts) o = *opts;
  o.solver = HUB_CG_FP64;
  if ((s = check_opts(o))) return s;
  std::lock_guard<std::mutex> lk(ctx->mu);
  HUB_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  const Geom g = make_geom(*lat);
  const size_t N = (size_t)g.n;
  const TileGeo tg = tile_geo(g, kSitesPerThread);
  const int nt = tg.ntiles;
  int bi = 0;
  for (int k = 1; k < nshift; ++k)
    if (mu2[k] < mu2[bi]) bi = k;
  const int ns = nshift - 1;
  const int maxit = o.max_iter;
  // workspace: r, p pair, u, the shifted directions, partials, scalars, descriptor, Lanczos history
  const size_t vecs = (size_t)(5 + ns) * N * 16;  // r, p pair, u, the phase, shifted directions
  const size_t parts = 2 * (size_t)nt * sizeof(double);
  const size_t hist_bytes = (2 * (size_t)maxit + 2) * sizeof(double);
  const size_t tail = ((sizeof(MsScal) + 255) / 256) * 256 + ((sizeof(MsDesc) + 255) / 256) * 256;
  char* ws = (char*)ctx->pool->alloc(vecs + parts + tail + hist_bytes, stream);
  if (!ws) return fail(HUB_ERR_OOM, "multi-shift workspace");
  double2* v = (double2*)ws;
  MsDesc h;
  std::memset(&h, 0, sizeof(h));
  h.g = g;
  h.ph64 = v + (size_t)(4 + ns) * N;
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
  h.tnb = tg.nb;
  h.tbsz = tg.bsz;
  h.tseg = tg.seg;
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
    hipError_t e = launch_phase(phi, const_cast<double2*>(h.ph64), nullptr, (int)N, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dd, &h, sizeof(h), hipMemcpyHostToDevice, stream);
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
    sys[k].phi = phi;
    sys[k].mu2 = mu2[k];
    sys[k].b = (const double2*)b;
    sys[k].x = (double2*)x + (size_t)k * N;
  }
  hub_solve_opts oc = o;
  oc.use_x0 = 1;
  result = run_solves(ctx, sys, oc, stream);
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

}  // extern "C"
