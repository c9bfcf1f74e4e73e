// The staggered-mass Hasenbusch split (hub_hasenbusch_heatbath, hub_hasenbusch_force)
// and HMC updates (hub_md_schedule, hub_hmc_trajectory, hub_hmc_trajectories).
//
// Everything is written over "chains": independent fields phi with their own
// pseudofermions.  A Hasenbusch call is one chain; hub_hmc_trajectories advances
// several Markov chains through the same molecular-dynamics schedule in lockstep,
// so each kick group solves the selected terms of every chain in one batch (the
// systems of all chains share the solver's launches).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "hub_api_internal.h"
#include "hub_md.h"

using namespace hub;
using namespace hub::api;

static_assert(HUB_MAX_HB_MASSES + 1 == kMaxLevels, "Hasenbusch levels");
static_assert(HUB_MAX_HB_MASSES + 1 <= kMaxSys, "one batched solve per term");
static_assert(sizeof(hub_hmc_params) == 232 && sizeof(hub_md_op) == 152 && sizeof(hub_hmc_info) == 120,
              "HMC struct layouts");

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

// The buffers of one chain (device unless noted).
struct Chain {
  const double* phi = nullptr;
  const double2* rho = nullptr;   // heat-bath vectors [n+1][N]
  double2* chi = nullptr;         // pseudofermions [n+1][N]
  double2* eta = nullptr;         // solutions per term [n+1][N]
  double* dS = nullptr;           // force accumulator [N] or NULL
  double* S = nullptr;            // host [n+1] or NULL
  hub_solve_info* info = nullptr; // host (heat-bath: [n]; evaluation: [n+1]) or NULL
};

// Heat-bath of the n+1 pseudofermions of every chain (Sec. 5.1):
//   chi_n = M_{n-1} rho_n,  chi_i = M_i^{-1} M_{i-1} rho_i = M_i^dag (M_i M_i^dag)^{-1} M_{i-1} rho_i.
// Caller holds ctx->mu, device set.  Synchronises the stream.
hub_status heatbath_impl(hub_ctx* ctx, const hub_lattice& lat, const double* mt, int n, std::vector<Chain>& ch,
                         const hub_solve_opts& o, hipStream_t stream) {
  const size_t N = (size_t)make_geom(lat).n;
  const int C = (int)ch.size();
  for (const Chain& c : ch)
    HUB_HIP(launch_apply(geom_with_mass(lat, mt, n - 1), c.phi, c.rho + n * N, c.chi + n * N, 1, false, stream),
            "apply");
  if (n == 0) HUB_HIP(hipStreamSynchronize(stream), "heat-bath");
  if (n == 0) return HUB_OK;
  double2* w = (double2*)ctx->pool->alloc(2 * (size_t)C * n * N * 16, stream);
  if (!w) return fail(HUB_ERR_OOM, "heat-bath workspace");
  double2* y = w + (size_t)C * n * N;
  std::vector<System> sys((size_t)C * n);
  hipError_t e = hipSuccess;
  for (int c = 0; c < C && e == hipSuccess; ++c)
    for (int i = 0; i < n && e == hipSuccess; ++i) {
      const size_t k = (size_t)c * n + i;
      e = launch_apply(geom_with_mass(lat, mt, i - 1), ch[c].phi, ch[c].rho + i * N, w + k * N, 1, false, stream);
      sys[k].g = geom_with_mass(lat, mt, i);
      sys[k].phi = ch[c].phi;
      sys[k].mu2 = 0.0;
      sys[k].b = w + k * N;
      sys[k].x = y + k * N;
    }
  hub_solve_opts oz = o;
  oz.use_x0 = 0;
  hub_status result = e == hipSuccess ? run_solves(ctx, sys, oz, stream) : hip_fail(e, "apply");
  if (result == HUB_OK || result == HUB_ERR_NOCONV) {
    for (int c = 0; c < C && e == hipSuccess; ++c)
      for (int i = 0; i < n && e == hipSuccess; ++i) {
        const size_t k = (size_t)c * n + i;
        e = launch_apply(sys[k].g, ch[c].phi, y + k * N, ch[c].chi + i * N, 1, true, stream);
      }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) result = hip_fail(e, "apply");
    for (int c = 0; c < C; ++c)
      if (ch[c].info)
        for (int i = 0; i < n; ++i) ch[c].info[i] = sys[(size_t)c * n + i].info;
  }
  ctx->pool->release(w, stream);
  return result;
}

// Actions and force of the selected terms of every chain (Sec. 5.1, eq. (f_chi_i)).
// Term terms[k] enters the chain's dS with scales[k] (dS untouched where NULL);
// S and info are indexed by term.  Caller holds ctx->mu, device set.  Synchronises.
hub_status eval_impl(hub_ctx* ctx, const hub_lattice& lat, const double* mt, int n, std::vector<Chain>& ch,
                     const std::vector<int>& terms, const std::vector<double>& scales, int accumulate,
                     const hub_solve_opts& o, hipStream_t stream) {
  const Geom g = make_geom(lat);
  const size_t N = (size_t)g.n;
  const int T = (int)terms.size();
  const int C = (int)ch.size();
  const int nt = ntiles_of(g.n);
  const size_t CT = (size_t)C * T;
  // workspace: M_i chi_i for the ratio terms and xi, per (chain, term); dot partials and results
  const size_t vec_bytes = CT * N * 16;
  const size_t part_bytes = CT * nt * sizeof(double);
  const size_t res_bytes = ((CT * sizeof(double) + 255) / 256) * 256;
  char* ws = (char*)ctx->pool->alloc(2 * vec_bytes + part_bytes + res_bytes, stream);
  if (!ws) return fail(HUB_ERR_OOM, "Hasenbusch workspace");
  double2* wv = (double2*)ws;
  double2* xv = (double2*)(ws + vec_bytes);
  double* part = (double*)(ws + 2 * vec_bytes);
  double* res = (double*)(ws + 2 * vec_bytes + part_bytes);
  std::vector<System> sys(CT);
  std::vector<const double2*> rhs(CT);
  hipError_t e = hipSuccess;
  for (int c = 0; c < C && e == hipSuccess; ++c)
    for (int k = 0; k < T && e == hipSuccess; ++k) {
      const size_t q = (size_t)c * T + k;
      const int i = terms[k];
      const int den = i == n ? n - 1 : i - 1;
      if (i == n) {
        rhs[q] = ch[c].chi + i * N;
      } else {
        e = launch_apply(geom_with_mass(lat, mt, i), ch[c].phi, ch[c].chi + i * N, wv + q * N, 1, false, stream);
        rhs[q] = wv + q * N;
      }
      sys[q].g = geom_with_mass(lat, mt, den);
      sys[q].phi = ch[c].phi;
      sys[q].mu2 = 0.0;
      sys[q].b = rhs[q];
      sys[q].x = ch[c].eta + i * N;
    }
  hub_status result = e == hipSuccess ? run_solves(ctx, sys, o, stream) : hip_fail(e, "apply");
  if (result == HUB_OK || result == HUB_ERR_NOCONV) {
    std::vector<double> Sh(CT, 0.0);
    for (int c = 0; c < C && e == hipSuccess; ++c)
      for (int k = 0; k < T && e == hipSuccess; ++k) {
        const size_t q = (size_t)c * T + k;
        const int i = terms[k];
        double2* et = ch[c].eta + i * N;
        // S_i = Re rhs_i^dag eta_i; xi_i = M_den^dag eta_i; dS_i/dphi with xi_i (- chi_i)
        e = launch_dot_re(g, rhs[q], et, 1, part + q * nt, res + q, stream);
        if (e == hipSuccess) e = launch_apply(sys[q].g, ch[c].phi, et, xv + q * N, 1, true, stream);
        if (e == hipSuccess && ch[c].dS)
          e = launch_force(g, ch[c].phi, et, xv + q * N, scales[k], (k == 0) ? accumulate : 1, ch[c].dS, 1,
                           stream, i == n ? nullptr : ch[c].chi + i * N);
      }
    if (e == hipSuccess) e = hipMemcpyAsync(Sh.data(), res, CT * sizeof(double), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      result = hip_fail(e, "Hasenbusch force");
    } else {
      for (int c = 0; c < C; ++c)
        for (int k = 0; k < T; ++k) {
          if (ch[c].S) ch[c].S[terms[k]] = Sh[(size_t)c * T + k];
          if (ch[c].info) ch[c].info[terms[k]] = sys[(size_t)c * T + k].info;
        }
    }
  }
  ctx->pool->release(ws, stream);
  return result;
}

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


// One HMC update of C chains in lockstep (Sec. 2, Sec. 5.2).  phi, pi: [C][N];
// rho: [C][n+1][N]; u, info: host [C].  Caller holds ctx->mu, device set.
hub_status hmc_impl(hub_ctx* ctx, const hub_lattice& lat, int C, double* phi, double* pi, const hub_c128* rho,
                    const double* u, const hub_hmc_params* params, const MdSchedule& sched,
                    const hub_solve_opts& o, hub_hmc_info* info, hipStream_t stream) {
  const int n = params->n;
  const double* mt = params->mt;
  const Geom g = make_geom(lat);
  const size_t N = (size_t)g.n;
  const int nt2 = ntiles_of(g.n / 2);
  for (int c = 0; c < C; ++c) std::memset(&info[c], 0, sizeof(hub_hmc_info));
  // workspace: phi at the start (rejections), the summed pseudofermion force G, chi and
  // eta per term, dot partials and results, for every chain
  const size_t fld = (size_t)C * N * sizeof(double), vec = (size_t)C * (n + 1) * N * 16;
  const size_t part_bytes = 2 * (size_t)C * nt2 * sizeof(double);
  const size_t res_bytes = ((2 * (size_t)C * sizeof(double) + 255) / 256) * 256;
  char* ws = (char*)ctx->pool->alloc(2 * fld + 2 * vec + part_bytes + res_bytes, stream);
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
  std::vector<std::vector<double>> S(C, std::vector<double>(n + 1, 0.0)), S0 = S;
  std::vector<std::vector<hub_solve_info>> sinfo(C, std::vector<hub_solve_info>(n + 1));
  std::vector<Chain> ch(C);
  for (int c = 0; c < C; ++c) {
    ch[c].phi = phi + c * N;
    ch[c].rho = (const double2*)rho + (size_t)c * (n + 1) * N;
    ch[c].chi = chi + (size_t)c * (n + 1) * N;
    ch[c].eta = eta + (size_t)c * (n + 1) * N;
    ch[c].S = S[c].data();
    ch[c].info = sinfo[c].data();
  }
  // phi^2 / (2 U~) and pi^2 / 2 per chain through the complex dot kernel on (re, im) pairs (N is even)
  Geom gh = g;
  gh.n = g.n / 2;
  std::vector<double> gauge(C), kin(C), gauge1(C), kin1(C);
  auto quadratic = [&](std::vector<double>& gs, std::vector<double>& ks) {
    std::vector<double> h(2 * (size_t)C);
    for (int c = 0; c < C; ++c) {
      const double2* pc = (const double2*)(phi + c * N);
      const double2* qc = (const double2*)(pi + c * N);
      if (!hip_check(launch_dot_re(gh, pc, pc, 1, part + (size_t)(2 * c) * nt2, res + 2 * c, stream), "norm"))
        return false;
      if (!hip_check(launch_dot_re(gh, qc, qc, 1, part + (size_t)(2 * c + 1) * nt2, res + 2 * c + 1, stream),
                     "norm"))
        return false;
    }
    if (!hip_check(hipMemcpyAsync(h.data(), res, h.size() * sizeof(double), hipMemcpyDeviceToHost, stream), "norm"))
      return false;
    if (!hip_check(hipStreamSynchronize(stream), "norm")) return false;
    for (int c = 0; c < C; ++c) {
      gs[c] = 0.5 * h[2 * c] / params->U_t;
      ks[c] = 0.5 * h[2 * c + 1];
    }
    return true;
  };
  std::vector<int> all(n + 1);
  for (int i = 0; i <= n; ++i) all[i] = i;
  bool evaluated = false;  // every term of every chain has a solution in eta (warm starts allowed)
  auto evaluate = [&](const std::vector<int>& terms, const std::vector<double>& scales, bool force) {
    hub_solve_opts oe = o;
    if (!evaluated) oe.use_x0 = 0;
    for (int c = 0; c < C; ++c) ch[c].dS = force ? G + c * N : nullptr;
    const hub_status st = eval_impl(ctx, lat, mt, n, ch, terms, scales, 0, oe, stream);
    if (st != HUB_OK) {
      if (result == HUB_OK) result = st;
      return false;
    }
    evaluated = evaluated || terms.size() == (size_t)(n + 1);
    for (int c = 0; c < C; ++c)
      for (int t : terms) {
        info[c].force_evals[t]++;
        info[c].inner_iters += sinfo[c][t].inner_iters;
      }
    return true;
  };
  auto all_levels = [&](const MdOp& op) {
    if (op.kind != 1) return false;
    for (int i = 0; i <= n; ++i)
      if (op.coef[i] == 0.0) return false;
    return true;
  };
  bool saved = false;
  do {
    if (!hip_check(hipMemcpyAsync(phi0, phi, fld, hipMemcpyDeviceToDevice, stream), "copy")) break;
    saved = true;
    if (params->flags & HUB_HMC_CHI_GIVEN) {
      if (!hip_check(hipMemcpyAsync(chi, rho, vec, hipMemcpyDeviceToDevice, stream), "copy")) break;
    } else {
      for (Chain& c : ch) c.info = nullptr;
      result = heatbath_impl(ctx, lat, mt, n, ch, o, stream);
      for (int c = 0; c < C; ++c) ch[c].info = sinfo[c].data();
      if (result != HUB_OK) break;
    }
    if (!quadratic(gauge, kin)) break;
    // the pseudofermion actions at the start come from the first kick group's solves
    // (every level kicks there unless zeta = 0)
    const bool first_all = all_levels(sched.ops.front());
    if (!first_all) {
      if (!evaluate(all, std::vector<double>(n + 1, 0.0), false)) break;
      S0 = S;
    }
    bool ok = true;
    for (size_t k = 0; k < sched.ops.size() && ok; ++k) {
      const MdOp& op = sched.ops[k];
      if (op.kind == 0) {
        ok = hip_check(launch_md_drift(phi, pi, op.eps, (int)(C * N), stream), "drift");
        for (int c = 0; c < C; ++c) info[c].drifts++;
        continue;
      }
      std::vector<int> terms;
      std::vector<double> scales;
      for (int l = 0; l <= n; ++l)
        if (op.coef[l] != 0.0) {
          terms.push_back(l);
          scales.push_back(op.coef[l]);
        }
      ok = evaluate(terms, scales, true);
      if (!ok) break;
      if (k == 0 && first_all) S0 = S;
      // pi -= sum_l coef_l dS_l/dphi + coef_n phi / U~ (the gauge force rides with level n)
      ok = hip_check(launch_md_kick(pi, phi, G, op.coef[n] / params->U_t, (int)(C * N), stream), "kick");
      for (int c = 0; c < C; ++c) info[c].kick_groups++;
    }
    if (!ok) break;
    if (!all_levels(sched.ops.back()) && !evaluate(all, std::vector<double>(n + 1, 0.0), false)) break;
    if (!quadratic(gauge1, kin1)) break;
  } while (false);
  if (result == HUB_OK) {
    for (int c = 0; c < C; ++c) {
      double sf0 = 0, sf1 = 0;
      for (int i = 0; i <= n; ++i) {
        sf0 += S0[c][i];
        sf1 += S[c][i];
      }
      info[c].H0 = gauge[c] + kin[c] + sf0;
      info[c].H1 = gauge1[c] + kin1[c] + sf1;
      info[c].dH = info[c].H1 - info[c].H0;
      info[c].accepted = (std::isfinite(info[c].dH) && u[c] < std::exp(-info[c].dH)) ? 1 : 0;
      if (!info[c].accepted)
        hip_check(hipMemcpyAsync(phi + c * N, phi0 + c * N, N * sizeof(double), hipMemcpyDeviceToDevice, stream),
                  "restore");
    }
    hip_check(hipStreamSynchronize(stream), "trajectory");
  } else if (saved) {
    // a failed update leaves phi as it was (best effort after a device error)
    if (hipMemcpyAsync(phi, phi0, fld, hipMemcpyDeviceToDevice, stream) == hipSuccess)
      (void)hipStreamSynchronize(stream);
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
  {
    const size_t nn = 2 * (size_t)lat->L1 * lat->L2 * lat->Nt, vb = (size_t)(n + 1) * nn * sizeof(hub_c128);
    if (overlaps(rho, vb, chi, vb) || overlaps(phi, nn * 8, chi, vb))
      return fail(HUB_ERR_ARG, "chi must not overlap rho or phi");
  }
  hub_solve_opts o;
  hub_default_opts(&o);
  if (opts) o = *opts;
  o.use_x0 = 0;
  if ((s = check_opts(o))) return s;
  std::lock_guard<std::mutex> lk(ctx->mu);
  HUB_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  std::vector<Chain> ch(1);
  ch[0].phi = phi;
  ch[0].rho = (const double2*)rho;
  ch[0].chi = (double2*)chi;
  ch[0].info = info;
  return heatbath_impl(ctx, *lat, mt, n, ch, o, stream);
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
  {
    const size_t nn = 2 * (size_t)lat->L1 * lat->L2 * lat->Nt, vb = (size_t)(n + 1) * nn * sizeof(hub_c128);
    if (overlaps(chi, vb, eta, vb) || overlaps(phi, nn * 8, eta, vb) || overlaps(dSdphi, nn * 8, eta, vb) ||
        overlaps(dSdphi, nn * 8, chi, vb) || overlaps(dSdphi, nn * 8, phi, nn * 8))
      return fail(HUB_ERR_ARG, "eta and dSdphi must not overlap each other, chi or phi");
  }
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
  std::vector<Chain> ch(1);
  ch[0].phi = phi;
  ch[0].chi = (double2*)chi;
  ch[0].eta = (double2*)eta;
  ch[0].dS = dSdphi;
  ch[0].S = S;
  ch[0].info = info;
  return eval_impl(ctx, *lat, mt, n, ch, terms, scales, accumulate, o, stream);
}

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


hub_status hub_hmc_trajectories(hub_ctx* ctx, const hub_lattice* lat, int32_t nchain, double* phi, double* pi,
                                const hub_c128* rho, const double* u, const hub_hmc_params* params,
                                const hub_solve_opts* opts, hub_hmc_info* info, hipStream_t stream) {
  set_error("");
  if (!ctx) return fail(HUB_ERR_ARG, "ctx is NULL");
  hub_status s = check_lattice(lat);
  if (s) return s;
  MdSchedule sched;
  if ((s = check_hmc(params, &sched))) return s;
  if (nchain < 1 || (long long)nchain * (params->n + 1) > HUB_MAX_BATCH)
    return fail(HUB_ERR_ARG, "nchain must be >= 1 with nchain * (n + 1) <= HUB_MAX_BATCH");
  if (!phi || !pi || !rho || !u || !info) return fail(HUB_ERR_ARG, "NULL buffer");
  {
    const size_t nn = 2 * (size_t)lat->L1 * lat->L2 * lat->Nt, fb = (size_t)nchain * nn * 8;
    const size_t rb = (size_t)nchain * (params->n + 1) * nn * sizeof(hub_c128);
    if (overlaps(phi, fb, pi, fb) || overlaps(phi, fb, rho, rb) || overlaps(pi, fb, rho, rb))
      return fail(HUB_ERR_ARG, "phi, pi and rho must not overlap");
  }
  for (int c = 0; c < nchain; ++c)
    if (!is_finite(u[c]) || u[c] < 0.0 || u[c] > 1.0) return fail(HUB_ERR_ARG, "u must be in [0, 1]");
  hub_solve_opts o;
  hub_default_opts(&o);
  if (opts) o = *opts;
  if ((s = check_opts(o))) return s;
  std::lock_guard<std::mutex> lk(ctx->mu);
  HUB_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  return hmc_impl(ctx, *lat, nchain, phi, pi, rho, u, params, sched, o, info, stream);
}

hub_status hub_hmc_trajectory(hub_ctx* ctx, const hub_lattice* lat, double* phi, double* pi, const hub_c128* rho,
                              double u, const hub_hmc_params* params, const hub_solve_opts* opts,
                              hub_hmc_info* info, hipStream_t stream) {
  return hub_hmc_trajectories(ctx, lat, 1, phi, pi, rho, &u, params, opts, info, stream);
}

}  // extern "C"
