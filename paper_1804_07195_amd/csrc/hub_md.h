// Molecular-dynamics schedule of one HMC trajectory (host code, no device calls).
//
// Sec. 5.2: the second-order Omelyan integrator with the momentum updates on the
// outside, T(h) = T_F(zeta h) T_pi(h/2) T_F((1-2 zeta) h) T_pi(h/2) T_F(zeta h),
// nested over time scales.  Level k < n kicks with the force of Hasenbusch term k,
// level n with the gauge force plus term n, and only level n moves phi.  A level-k
// step is N_k innermost steps long (N_n = 1); each of its two T_pi(h/2) is the
// integration of level k+1 over h/2, i.e. N_k / (2 N_{k+1}) level-(k+1) steps.  For
// an odd ratio the level-(k+1) step next to the middle kick is cut in half through
// its own middle kick:
//   before the middle: T_F(zeta h') T_pi-part(h'/2) T_F((1-2 zeta) h'/2)
//   after the middle:  T_F((1-2 zeta) h'/2) T_pi-part(h'/2) T_F(zeta h')
//
// The schedule is emitted as a list of operations in which every run of
// consecutive kicks (all at the same phi) is merged into one kick group holding a
// coefficient per level: the device then solves for all the levels of a group in
// one batch.  Kicks with a zero coefficient (zeta = 0, the leapfrog) are dropped
// and consecutive drifts are merged.
#pragma once

#include <cmath>
#include <string>
#include <vector>

namespace hub {

constexpr int kMaxLevels = 17;  // HUB_MAX_HB_MASSES + 1

struct MdOp {
  int kind = 0;            // 0: drift phi += eps pi;  1: kick group pi -= sum_k coef[k] dS_k/dphi
  double eps = 0.0;
  double coef[kMaxLevels] = {0.0};
};

class MdSchedule {
 public:
  // n: Hasenbusch masses (levels 0..n); N[0..n-1]: innermost steps per level-k step.
  bool build(int n, const int* N, int n_md, double t, double zeta, std::string* err) {
    ops.clear();
    if (n < 0 || n >= kMaxLevels) return bad(err, "number of levels out of range");
    if (n_md < 1) return bad(err, "n_md must be >= 1");
    if (!(t > 0.0) || !std::isfinite(t)) return bad(err, "trajectory length must be finite and > 0");
    if (!std::isfinite(zeta) || zeta < 0.0 || zeta > 0.5) return bad(err, "zeta must be in [0, 0.5]");
    n_ = n;
    zeta_ = zeta;
    ratio_.assign(n + 1, 1);
    std::vector<long> full(n + 1, 1);
    for (int k = 0; k < n; ++k) {
      if (N[k] < 1) return bad(err, "time-scale factors must be >= 1");
      full[k] = N[k];
    }
    for (int k = 0; k < n; ++k) {
      if (full[k] % full[k + 1] != 0) return bad(err, "N_{k+1} must divide N_k");
      ratio_[k] = (int)(full[k] / full[k + 1]);
    }
    if (n > 0 && n_md % full[0] != 0) return bad(err, "N_0 must divide n_md");
    const double dt = t / n_md;
    h_.assign(n + 1, dt);
    for (int k = 0; k < n; ++k) h_[k] = dt * (double)full[k];
    const long outer = n > 0 ? n_md / full[0] : n_md;
    for (long s = 0; s < outer; ++s) step(0, h_[0]);
    return true;
  }

  std::vector<MdOp> ops;

 private:
  static bool bad(std::string* err, const char* m) {
    if (err) *err = m;
    return false;
  }
  void kick(int level, double e) {
    if (e == 0.0) return;
    if (ops.empty() || ops.back().kind != 1) {
      MdOp o;
      o.kind = 1;
      ops.push_back(o);
    }
    ops.back().coef[level] += e;
  }
  void drift(double e) {
    if (!ops.empty() && ops.back().kind == 0) {
      ops.back().eps += e;
      return;
    }
    MdOp o;
    o.kind = 0;
    o.eps = e;
    ops.push_back(o);
  }
  void step(int k, double h) {
    kick(k, zeta_ * h);
    inner(k, h, true);
    kick(k, (1.0 - 2.0 * zeta_) * h);
    inner(k, h, false);
    kick(k, zeta_ * h);
  }
  // What fills one half (h/2) of a level-k step.
  void inner(int k, double h, bool before_middle) {
    if (k == n_) {
      drift(0.5 * h);
      return;
    }
    const int whole = ratio_[k] / 2;
    const bool cut = (ratio_[k] & 1) != 0;
    if (before_middle) {
      for (int s = 0; s < whole; ++s) step(k + 1, h_[k + 1]);
      if (cut) half_step(k + 1, h_[k + 1], true);
    } else {
      if (cut) half_step(k + 1, h_[k + 1], false);
      for (int s = 0; s < whole; ++s) step(k + 1, h_[k + 1]);
    }
  }
  void half_step(int k, double h, bool before_middle) {
    if (before_middle) {
      kick(k, zeta_ * h);
      inner(k, h, true);
      kick(k, 0.5 * (1.0 - 2.0 * zeta_) * h);
    } else {
      kick(k, 0.5 * (1.0 - 2.0 * zeta_) * h);
      inner(k, h, false);
      kick(k, zeta_ * h);
    }
  }

  int n_ = 0;
  double zeta_ = 0.0;
  std::vector<int> ratio_;
  std::vector<double> h_;
};

}  // namespace hub
