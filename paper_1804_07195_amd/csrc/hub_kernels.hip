// HIP kernels for CDNA4 (gfx950): the honeycomb fermion operator of eq. (ferm_op),
// its adjoint, the normal operator M M^dagger + mu^2 (Sec. 3, Sec. 5.1), the fused
// conjugate-gradient iteration in FP64 and complex64, the Krylov helpers of the
// flexible GMRES of Appendix A, and the pseudofermion force of eqs. (p_dot), (eta_xi).
//
// Design (memory-bound stencil, no dense contraction, so no MFMA):
// * one thread per site, kSitesPerThread sites per thread, site-major layout with
//   j fastest so every neighbour stream is a coalesced, shifted copy of the own stream;
//   the neighbour index is computed from the site coordinates, never stored;
// * workgroup ids are remapped so that each XCD walks a contiguous range of tiles and
//   the t +- 1 and i +- 1 neighbours of a tile are mostly in the same XCD's L2;
// * the CG iteration is two kernels: (1) p = r + beta p on the fly, u = M^dagger p,
//   <p, A p> = |u|^2 + mu^2 |p|^2; (2) q = M u + mu^2 p, x += alpha p, r -= alpha q,
//   |r|^2.  Scalars alpha, beta and the convergence flag never leave the device;
// * reductions are deterministic: wave64 butterfly, fixed LDS combine, one partial
//   per tile, and the last workgroup of each system sums the partials in a fixed
//   order.  Results depend only on the system's own shape, not on the batch.
#include "hub_internal.h"

namespace hub {
namespace {

template <typename R> struct V2;
template <> struct V2<double> { using T = double2; };
template <> struct V2<float> { using T = float2; };

__device__ __forceinline__ void phase_cs(double ph, double& c, double& s) { sincos(ph, &s, &c); }
__device__ __forceinline__ void phase_cs(float ph, float& c, float& s) { sincosf(ph, &s, &c); }

// Workgroups are dispatched round-robin over the XCDs; give XCD x the x-th
// contiguous chunk of logical tiles.
__device__ __forceinline__ int xcd_remap(int b, int G) {
  const int per = G / kNumXcd, rem = G % kNumXcd;
  const int x = b % kNumXcd, k = b / kNumXcd;
  return (x < rem) ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
}

template <typename C> __device__ __forceinline__ C cz() { C z; z.x = 0; z.y = 0; return z; }

template <typename R, typename C>
__device__ __forceinline__ R norm2(C a) { return a.x * a.x + a.y * a.y; }

// The stencil of M (DAG = false) or M^dagger (DAG = true) at site n.
//   M,  A row: -x(n) + s (e^{ i phi(n)}  - m) x(t-1) - kappa sum_bonds x_B
//   M,  B row: +x(n) - s (e^{-i phi(n)}  - m) x(t+1) - kappa sum_bonds x_A
//   M+, A row: -x(n) + s (e^{-i phi(tn)} - m) x(t+1) - kappa sum_bonds x_B
//   M+, B row: +x(n) - s (e^{ i phi(tn)} - m) x(t-1) - kappa sum_bonds x_A
// with s = -1 on a hop across the antiperiodic temporal boundary.  `ld(k)` returns
// the input vector at site k; the own-site value is returned in `self`.
template <typename R, bool DAG, typename PhiT, typename Load>
__device__ __forceinline__ typename V2<R>::T stencil(const Geom& g, const PhiT* __restrict__ phi, int n,
                                                     Load ld, typename V2<R>::T& self) {
  using C = typename V2<R>::T;
  const uint32_t q1 = fdiv((uint32_t)n, g.dL2);
  const int j = n - (int)q1 * g.L2;
  const uint32_t q2 = fdiv(q1, g.dL1);
  const int i = (int)q1 - (int)q2 * g.L1;
  const bool isA = (q2 & 1u) == 0;
  const int t = (int)(q2 >> 1);
  const int P2 = 2 * g.P;
  const bool fwd = (isA == DAG);
  int tn;
  R sgn;
  if (fwd) {
    const bool wrap = t == g.Nt - 1;
    tn = wrap ? n - (g.Nt - 1) * P2 : n + P2;
    sgn = wrap ? R(-1) : R(1);
  } else {
    const bool wrap = t == 0;
    tn = wrap ? n + (g.Nt - 1) * P2 : n - P2;
    sgn = wrap ? R(-1) : R(1);
  }
  int h0, h1, h2;
  if (isA) {
    const int b = n + g.P;
    h0 = b;
    h1 = (i > 0) ? b - g.L2 : b + (g.L1 - 1) * g.L2;
    h2 = (j > 0) ? b - 1 : b + g.L2 - 1;
  } else {
    const int a = n - g.P;
    h0 = a;
    h1 = (i < g.L1 - 1) ? a + g.L2 : a - (g.L1 - 1) * g.L2;
    h2 = (j < g.L2 - 1) ? a + 1 : a - (g.L2 - 1);
  }
  const C xs = ld(n);
  const C xt = ld(tn);
  const C x0 = ld(h0);
  const C x1 = ld(h1);
  const C x2 = ld(h2);
  R c, s;
  phase_cs((R)phi[DAG ? tn : n], c, s);
  const R es = (isA != DAG) ? s : -s;          // e^{+i phi} iff A row of M or B row of M^dagger
  const R cr = sgn * (c - (R)g.ms), ci = sgn * es;
  const R tr = cr * xt.x - ci * xt.y, ti = cr * xt.y + ci * xt.x;
  const R sig = isA ? R(-1) : R(1);
  const R kap = (R)g.kappa;
  C y;
  y.x = sig * (xs.x - tr) - kap * (x0.x + x1.x + x2.x);
  y.y = sig * (xs.y - ti) - kap * (x0.y + x1.y + x2.y);
  self = xs;
  return y;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic sum over the 256 threads; every thread gets the same value.
template <typename T>
__device__ __forceinline__ T block_sum(T v) {
  __shared__ T lds[kBlock / 64];
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  return (lds[0] + lds[1]) + (lds[2] + lds[3]);
}

// Publish this tile's `nv` block totals; the workgroup that finishes last sums all
// tiles' partials in a fixed order into `out` (valid in every thread of that
// workgroup) and returns true.  Resets the counter for the next reduction.
__device__ bool finish_reduction(const double* vals, int nv, double* part, unsigned* counter, int ntiles,
                                 int tile, double* out) {
  __shared__ int s_last;
  if (threadIdx.x == 0) {
    for (int q = 0; q < nv; ++q)
      __hip_atomic_store(&part[(size_t)tile * kMaxRed + q], vals[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    s_last = (prev == (unsigned)(ntiles - 1));
  }
  __syncthreads();
  if (!s_last) return false;
  __threadfence();
  for (int q = 0; q < nv; ++q) {
    double acc = 0.0;
    for (int k = threadIdx.x; k < ntiles; k += kBlock)
      acc += __hip_atomic_load(&part[(size_t)k * kMaxRed + q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const double tot = block_sum(acc);
    if (threadIdx.x == 0) out[q] = tot;
  }
  if (threadIdx.x == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  return true;
}

__device__ __forceinline__ int find_sys(const LaunchList& L, int lt) {
  int lo = 0, hi = L.nsys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (L.tile_begin[mid] <= lt) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename PhiT> __device__ __forceinline__ const PhiT* phi_of(const SysDesc* d);
template <> __device__ __forceinline__ const double* phi_of<double>(const SysDesc* d) { return d->phi; }
template <> __device__ __forceinline__ const float* phi_of<float>(const SysDesc* d) { return d->phi32; }

// ---------------------------------------------------------------------------
// Public operator kernels (shared phi, batch of vectors, no descriptors).
// ---------------------------------------------------------------------------
template <bool DAG>
__global__ __launch_bounds__(kBlock) void k_apply(Geom g, const double* __restrict__ phi,
                                                  const double2* __restrict__ x, double2* __restrict__ y,
                                                  int ntiles) {
  const int l = xcd_remap(blockIdx.x, gridDim.x);
  const int b = l / ntiles, tile = l - b * ntiles;
  const double2* __restrict__ xb = x + (size_t)b * g.n;
  double2* __restrict__ yb = y + (size_t)b * g.n;
  const int base = tile * kTile + threadIdx.x;
  auto ld = [=](int k) { return xb[k]; };
#pragma unroll
  for (int m = 0; m < kSitesPerThread; ++m) {
    const int n = base + m * kBlock;
    if (n < g.n) {
      double2 self;
      yb[n] = stencil<double, DAG>(g, phi, n, ld, self);
    }
  }
}

struct Mu2Arr { double v[kMaxSys]; };

__global__ __launch_bounds__(kBlock) void k_normal2_pub(Geom g, const double* __restrict__ phi, Mu2Arr mu2,
                                                        const double2* __restrict__ u,
                                                        const double2* __restrict__ x, double2* __restrict__ y,
                                                        int ntiles) {
  const int l = xcd_remap(blockIdx.x, gridDim.x);
  const int b = l / ntiles, tile = l - b * ntiles;
  const size_t off = (size_t)b * g.n;
  const double m2 = mu2.v[b];
  const int base = tile * kTile + threadIdx.x;
  auto ld = [=](int k) { return u[off + k]; };
#pragma unroll
  for (int m = 0; m < kSitesPerThread; ++m) {
    const int n = base + m * kBlock;
    if (n < g.n) {
      double2 self;
      double2 q = stencil<double, false>(g, phi, n, ld, self);
      const double2 xv = x[off + n];
      q.x += m2 * xv.x;
      q.y += m2 * xv.y;
      y[off + n] = q;
    }
  }
}

// dS/dphi at every site: A: 2 Im[conj(eta(t)) s e^{i phi} xi(t-1)],
//                        B: 2 Im[conj(eta(t)) s e^{-i phi} xi(t+1)].
__global__ __launch_bounds__(kBlock) void k_force(Geom g, const double* __restrict__ phi,
                                                  const double2* __restrict__ eta,
                                                  const double2* __restrict__ xi, double scale, int accumulate,
                                                  double* __restrict__ out, int ntiles) {
  const int l = xcd_remap(blockIdx.x, gridDim.x);
  const int b = l / ntiles, tile = l - b * ntiles;
  const size_t off = (size_t)b * g.n;
  const int base = tile * kTile + threadIdx.x;
  const int P2 = 2 * g.P;
#pragma unroll
  for (int m = 0; m < kSitesPerThread; ++m) {
    const int n = base + m * kBlock;
    if (n < g.n) {
      const uint32_t q2 = fdiv(fdiv((uint32_t)n, g.dL2), g.dL1);
      const bool isA = (q2 & 1u) == 0;
      const int t = (int)(q2 >> 1);
      int tn;
      double sgn;
      if (isA) {
        const bool wrap = t == 0;
        tn = wrap ? n + (g.Nt - 1) * P2 : n - P2;
        sgn = wrap ? -1.0 : 1.0;
      } else {
        const bool wrap = t == g.Nt - 1;
        tn = wrap ? n - (g.Nt - 1) * P2 : n + P2;
        sgn = wrap ? -1.0 : 1.0;
      }
      double c, s;
      sincos(phi[n], &s, &c);
      if (!isA) s = -s;
      const double2 e = eta[off + n], z = xi[off + tn];
      // w = s*(c + i s) * z ; F = 2 Im(conj(e) * w)
      const double wr = sgn * (c * z.x - s * z.y), wi = sgn * (c * z.y + s * z.x);
      const double F = 2.0 * (e.x * wi - e.y * wr);
      double* o = out + off + n;
      *o = accumulate ? *o + scale * F : scale * F;
    }
  }
}

// result[b] = Re sum conj(a_b) b_b, deterministic per b.
__global__ __launch_bounds__(kBlock) void k_dot_re(Geom g, const double2* __restrict__ a,
                                                   const double2* __restrict__ bb, int ntiles, double* part,
                                                   unsigned* counters, double* result) {
  const int l = xcd_remap(blockIdx.x, gridDim.x);
  const int b = l / ntiles, tile = l - b * ntiles;
  const size_t off = (size_t)b * g.n;
  const int base = tile * kTile + threadIdx.x;
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < kSitesPerThread; ++m) {
    const int n = base + m * kBlock;
    if (n < g.n) {
      const double2 u = a[off + n], v = bb[off + n];
      acc += u.x * v.x + u.y * v.y;
    }
  }
  double tot = block_sum(acc);
  double out;
  if (finish_reduction(&tot, 1, part + (size_t)b * ntiles * kMaxRed, counters + b, ntiles, tile, &out)) {
    if (threadIdx.x == 0) result[b] = out;
  }
}

__global__ __launch_bounds__(kBlock) void k_phi_to_f32(const double* __restrict__ phi, float* __restrict__ p32,
                                                       int n) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p32[i] = (float)phi[i];
}

// ---------------------------------------------------------------------------
// Batched solver kernels (descriptor + launch list).
// ---------------------------------------------------------------------------
#define HUB_PROLOGUE                                   \
  const int lt = xcd_remap(blockIdx.x, gridDim.x);     \
  const int kk = find_sys(L, lt);                      \
  const SysDesc* __restrict__ d = sys + L.sys[kk];     \
  const int tile = lt - L.tile_begin[kk];              \
  Scal* sc = d->sc;                                    \
  const Geom g = d->g;                                 \
  const int base = tile * kTile + threadIdx.x;

// CG stage 1: p_new = r + beta p_old (p_new = r on a fresh start), u = M^dagger p_new,
// alpha = rr / (|u|^2 + mu^2 |p_new|^2).
template <typename R, typename PhiT>
__global__ __launch_bounds__(kBlock) void k_cg1(const SysDesc* __restrict__ sys, LaunchList L, int sR, int sP,
                                                int sU) {
  using C = typename V2<R>::T;
  HUB_PROLOGUE
  if (!sc->active) return;
  const int it = sc->iters;
  const bool fresh = sc->fresh != 0;
  const R beta = (R)sc->beta;
  const R mu2 = (R)d->mu2;
  const C* __restrict__ r = (const C*)d->vec[sR];
  const C* __restrict__ po = (const C*)d->vec[sP + (it & 1)];
  C* __restrict__ pn = (C*)d->vec[sP + 1 - (it & 1)];
  C* __restrict__ u = (C*)d->vec[sU];
  const PhiT* __restrict__ phi = phi_of<PhiT>(d);
  R acc = 0;
  if (fresh) {
    auto ld = [=](int k) { return r[k]; };
#pragma unroll
    for (int m = 0; m < kSitesPerThread; ++m) {
      const int n = base + m * kBlock;
      if (n < g.n) {
        C p;
        const C uu = stencil<R, true>(g, phi, n, ld, p);
        pn[n] = p;
        u[n] = uu;
        acc += norm2<R>(uu) + mu2 * norm2<R>(p);
      }
    }
  } else {
    auto ld = [=](int k) {
      const C a = r[k], b = po[k];
      C o;
      o.x = a.x + beta * b.x;
      o.y = a.y + beta * b.y;
      return o;
    };
#pragma unroll
    for (int m = 0; m < kSitesPerThread; ++m) {
      const int n = base + m * kBlock;
      if (n < g.n) {
        C p;
        const C uu = stencil<R, true>(g, phi, n, ld, p);
        pn[n] = p;
        u[n] = uu;
        acc += norm2<R>(uu) + mu2 * norm2<R>(p);
      }
    }
  }
  double tot = (double)block_sum(acc);
  double pq;
  if (finish_reduction(&tot, 1, d->part, d->counter, d->ntiles, tile, &pq)) {
    if (threadIdx.x == 0) sc->alpha = sc->rr / pq;
  }
}

// CG stage 2: q = M u + mu^2 p, x += alpha p, r -= alpha q; beta = |r|^2_new / |r|^2
// and the convergence flag.  The solution slot of system k is L.pi[k].
template <typename R, typename PhiT>
__global__ __launch_bounds__(kBlock) void k_cg2(const SysDesc* __restrict__ sys, LaunchList L, int sR, int sP,
                                                int sU) {
  using C = typename V2<R>::T;
  HUB_PROLOGUE
  if (!sc->active) return;
  const int it = sc->iters;
  const R alpha = (R)sc->alpha;
  const R mu2 = (R)d->mu2;
  const C* __restrict__ p = (const C*)d->vec[sP + 1 - (it & 1)];
  const C* __restrict__ u = (const C*)d->vec[sU];
  C* __restrict__ x = (C*)d->vec[L.pi[kk]];
  C* __restrict__ r = (C*)d->vec[sR];
  const PhiT* __restrict__ phi = phi_of<PhiT>(d);
  auto ld = [=](int k) { return u[k]; };
  R acc = 0;
#pragma unroll
  for (int m = 0; m < kSitesPerThread; ++m) {
    const int n = base + m * kBlock;
    if (n < g.n) {
      C self;
      C q = stencil<R, false>(g, phi, n, ld, self);
      const C pv = p[n];
      q.x += mu2 * pv.x;
      q.y += mu2 * pv.y;
      C xv = x[n], rv = r[n];
      xv.x += alpha * pv.x;
      xv.y += alpha * pv.y;
      rv.x -= alpha * q.x;
      rv.y -= alpha * q.y;
      x[n] = xv;
      r[n] = rv;
      acc += norm2<R>(rv);
    }
  }
  double tot = (double)block_sum(acc);
  double rr_new;
  if (finish_reduction(&tot, 1, d->part, d->counter, d->ntiles, tile, &rr_new)) {
    if (threadIdx.x == 0) {
      sc->beta = rr_new / sc->rr;
      sc->rr = rr_new;
      sc->iters = it + 1;
      sc->fresh = 0;
      if (!(rr_new > sc->stop2) || it + 1 >= sc->maxit) sc->active = 0;
    }
  }
}

template <typename Tin> __device__ __forceinline__ double2 to_c128(Tin v);
template <> __device__ __forceinline__ double2 to_c128<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ double2 to_c128<float2>(float2 v) {
  double2 o;
  o.x = v.x;
  o.y = v.y;
  return o;
}

// u = M^dagger in (FP64 arithmetic; in is FP64 or C64).
template <typename Tin>
__global__ __launch_bounds__(kBlock) void k_mdag_slot(const SysDesc* __restrict__ sys, LaunchList L, int s_in) {
  HUB_PROLOGUE
  (void)sc;
  const Tin* __restrict__ in = (const Tin*)d->vec[s_in];
  double2* __restrict__ u = (double2*)d->vec[S_U];
  auto ld = [=](int k) { return to_c128<Tin>(in[k]); };
#pragma unroll
  for (int m = 0; m < kSitesPerThread; ++m) {
    const int n = base + m * kBlock;
    if (n < g.n) {
      double2 self;
      u[n] = stencil<double, true>(g, d->phi, n, ld, self);
    }
  }
}

__device__ __forceinline__ void cg_setup(Scal* sc, double rr, double pa, double pr, int maxit) {
  sc->rr = rr;
  sc->stop2 = pa + pr * rr;
  sc->iters = 0;
  sc->maxit = maxit;
  sc->fresh = 1;
  sc->active = (rr > sc->stop2) ? 1 : 0;
}

// out = [b -] (M u + mu^2 in), |out|^2 reduced with the given epilogue.
template <typename Tin>
__global__ __launch_bounds__(kBlock) void k_normal2_slot(const SysDesc* __restrict__ sys, LaunchList L, int s_in,
                                                         int s_b, int s_out, int mode, int red_off) {
  HUB_PROLOGUE
  const Tin* __restrict__ in = (const Tin*)d->vec[s_in];
  const double2* __restrict__ bv = s_b >= 0 ? (const double2*)d->vec[s_b] : nullptr;
  const double2* __restrict__ u = (const double2*)d->vec[S_U];
  double2* __restrict__ out = (double2*)d->vec[s_out];
  const double mu2 = d->mu2;
  auto ld = [=](int k) { return u[k]; };
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < kSitesPerThread; ++m) {
    const int n = base + m * kBlock;
    if (n < g.n) {
      double2 self;
      double2 q = stencil<double, false>(g, d->phi, n, ld, self);
      const double2 xv = to_c128<Tin>(in[n]);
      q.x += mu2 * xv.x;
      q.y += mu2 * xv.y;
      if (bv) {
        const double2 b = bv[n];
        q.x = b.x - q.x;
        q.y = b.y - q.y;
      }
      out[n] = q;
      acc += norm2<double>(q);
    }
  }
  if (mode == RED_NONE) return;
  double tot = block_sum(acc);
  double res;
  if (finish_reduction(&tot, 1, d->part, d->counter, d->ntiles, tile, &res)) {
    if (threadIdx.x == 0) {
      sc->red[red_off] = res;
      if (mode == RED_CG_SETUP) cg_setup(sc, res, L.pa[kk], L.pr[kk], L.pi[kk]);
    }
  }
}

// x = 0, r = b; |b|^2 -> red[0] and the FP64 CG setup.
__global__ __launch_bounds__(kBlock) void k_cg_init_zero(const SysDesc* __restrict__ sys, LaunchList L) {
  HUB_PROLOGUE
  const double2* __restrict__ b = (const double2*)d->vec[S_B];
  double2* __restrict__ x = (double2*)d->vec[S_X];
  double2* __restrict__ r = (double2*)d->vec[S_R];
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < kSitesPerThread; ++m) {
    const int n = base + m * kBlock;
    if (n < g.n) {
      const double2 v = b[n];
      r[n] = v;
      x[n] = cz<double2>();
      acc += norm2<double>(v);
    }
  }
  double tot = block_sum(acc);
  double res;
  if (finish_reduction(&tot, 1, d->part, d->counter, d->ntiles, tile, &res)) {
    if (threadIdx.x == 0) {
      sc->red[0] = res;
      cg_setup(sc, res, L.pa[kk], L.pr[kk], L.pi[kk]);
    }
  }
}

// red[off + 2i], red[off + 2i + 1] = <v_i, w> = sum conj(v_i) w, i < cnt.
__global__ __launch_bounds__(kBlock) void k_multidot(const SysDesc* __restrict__ sys, LaunchList L, int s_w,
                                                     int s_v0, int cnt, int red_off) {
  HUB_PROLOGUE
  const double2* __restrict__ w = (const double2*)d->vec[s_w];
  double2 wv[kSitesPerThread];
#pragma unroll
  for (int m = 0; m < kSitesPerThread; ++m) {
    const int n = base + m * kBlock;
    wv[m] = n < g.n ? w[n] : cz<double2>();
  }
  __shared__ double tot[kMaxRed];
  for (int q = 0; q < cnt; ++q) {
    const double2* __restrict__ v = (const double2*)d->vec[s_v0 + q];
    double ar = 0.0, ai = 0.0;
#pragma unroll
    for (int m = 0; m < kSitesPerThread; ++m) {
      const int n = base + m * kBlock;
      if (n < g.n) {
        const double2 vv = v[n];
        ar += vv.x * wv[m].x + vv.y * wv[m].y;
        ai += vv.x * wv[m].y - vv.y * wv[m].x;
      }
    }
    const double sr = block_sum(ar);
    const double si = block_sum(ai);
    if (threadIdx.x == 0) {
      tot[2 * q] = sr;
      tot[2 * q + 1] = si;
    }
  }
  __syncthreads();
  __shared__ double res[kMaxRed];
  if (finish_reduction(tot, 2 * cnt, d->part, d->counter, d->ntiles, tile, res)) {
    if (threadIdx.x == 0)
      for (int q = 0; q < 2 * cnt; ++q) sc->red[red_off + q] = res[q];
  }
}

// w -= sum_i h_i v_i, h_i = red[h_off + 2i] + i red[h_off + 2i + 1]; |w|^2 -> red[red_off].
__global__ __launch_bounds__(kBlock) void k_cgs(const SysDesc* __restrict__ sys, LaunchList L, int s_w, int s_v0,
                                                int cnt, int h_off, int red_off) {
  HUB_PROLOGUE
  double2* __restrict__ w = (double2*)d->vec[s_w];
  double2 wv[kSitesPerThread];
#pragma unroll
  for (int m = 0; m < kSitesPerThread; ++m) {
    const int n = base + m * kBlock;
    wv[m] = n < g.n ? w[n] : cz<double2>();
  }
  for (int q = 0; q < cnt; ++q) {
    const double hr = sc->red[h_off + 2 * q], hi = sc->red[h_off + 2 * q + 1];
    const double2* __restrict__ v = (const double2*)d->vec[s_v0 + q];
#pragma unroll
    for (int m = 0; m < kSitesPerThread; ++m) {
      const int n = base + m * kBlock;
      if (n < g.n) {
        const double2 vv = v[n];
        wv[m].x -= hr * vv.x - hi * vv.y;
        wv[m].y -= hr * vv.y + hi * vv.x;
      }
    }
  }
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < kSitesPerThread; ++m) {
    const int n = base + m * kBlock;
    if (n < g.n) {
      w[n] = wv[m];
      acc += norm2<double>(wv[m]);
    }
  }
  double tot = block_sum(acc);
  double res;
  if (finish_reduction(&tot, 1, d->part, d->counter, d->ntiles, tile, &res)) {
    if (threadIdx.x == 0) sc->red[red_off] = res;
  }
}

// v = pa*src (FP64, stored to s_v if s_v >= 0).  With pi = maxit > 0 the
// single-precision CG starts on v: r32 = c64(v), z = 0, rr = |r32|^2 (FP32 sums),
// stop2 = pr*rr.  With pi = 0 there is no preconditioning: z = c64(v).  The z slot
// of system k is pj[k].
__global__ __launch_bounds__(kBlock) void k_prep_inner(const SysDesc* __restrict__ sys, LaunchList L, int s_src,
                                                       int s_v) {
  HUB_PROLOGUE
  const double scale = L.pa[kk];
  const int maxit = L.pi[kk];
  const double2* __restrict__ src = (const double2*)d->vec[s_src];
  double2* __restrict__ v = s_v >= 0 ? (double2*)d->vec[s_v] : nullptr;
  float2* __restrict__ z = (float2*)d->vec[L.pj[kk]];
  float2* __restrict__ r32 = (float2*)d->vec[S_R32];
  float acc = 0.0f;
#pragma unroll
  for (int m = 0; m < kSitesPerThread; ++m) {
    const int n = base + m * kBlock;
    if (n < g.n) {
      double2 a = src[n];
      a.x *= scale;
      a.y *= scale;
      if (v) v[n] = a;
      float2 a32;
      a32.x = (float)a.x;
      a32.y = (float)a.y;
      if (maxit > 0) {
        r32[n] = a32;
        z[n] = cz<float2>();
        acc += norm2<float>(a32);
      } else {
        z[n] = a32;
      }
    }
  }
  if (maxit <= 0) return;
  double tot = (double)block_sum(acc);
  double res;
  if (finish_reduction(&tot, 1, d->part, d->counter, d->ntiles, tile, &res)) {
    if (threadIdx.x == 0) cg_setup(sc, res, 0.0, L.pr[kk], maxit);
  }
}

// x = (set ? 0 : x) + sum_{i < cnt} y_i z_i, y from sc->y, z_i the C64 slot S_Z0 + i.
__global__ __launch_bounds__(kBlock) void k_xupdate(const SysDesc* __restrict__ sys, LaunchList L, int cnt,
                                                    int set) {
  HUB_PROLOGUE
  double2* __restrict__ x = (double2*)d->vec[S_X];
  double2 xv[kSitesPerThread];
#pragma unroll
  for (int m = 0; m < kSitesPerThread; ++m) {
    const int n = base + m * kBlock;
    xv[m] = (n < g.n && !set) ? x[n] : cz<double2>();
  }
  for (int q = 0; q < cnt; ++q) {
    const double yr = sc->y[2 * q], yi = sc->y[2 * q + 1];
    const float2* __restrict__ z = (const float2*)d->vec[S_Z0 + q];
#pragma unroll
    for (int m = 0; m < kSitesPerThread; ++m) {
      const int n = base + m * kBlock;
      if (n < g.n) {
        const float2 zf = z[n];
        const double zr = zf.x, zi = zf.y;
        xv[m].x += yr * zr - yi * zi;
        xv[m].y += yr * zi + yi * zr;
      }
    }
  }
#pragma unroll
  for (int m = 0; m < kSitesPerThread; ++m) {
    const int n = base + m * kBlock;
    if (n < g.n) x[n] = xv[m];
  }
}

}  // namespace
}  // namespace hub

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
namespace hub {

static inline int tiles_of(int n) { return (n + kTile - 1) / kTile; }

hipError_t launch_apply(const Geom& g, const double* phi, const double2* x, double2* y, int batch, bool dag,
                        hipStream_t st) {
  const int nt = tiles_of(g.n);
  const dim3 grid(nt * batch), block(kBlock);
  if (dag)
    hipLaunchKernelGGL(k_apply<true>, grid, block, 0, st, g, phi, x, y, nt);
  else
    hipLaunchKernelGGL(k_apply<false>, grid, block, 0, st, g, phi, x, y, nt);
  return hipGetLastError();
}

hipError_t launch_normal2(const Geom& g, const double* phi, const double mu2_host[kMaxSys], const double2* u,
                          const double2* x, double2* y, int batch, hipStream_t st) {
  const int nt = tiles_of(g.n);
  Mu2Arr m;
  for (int b = 0; b < kMaxSys; ++b) m.v[b] = b < batch ? mu2_host[b] : 0.0;
  hipLaunchKernelGGL(k_normal2_pub, dim3(nt * batch), dim3(kBlock), 0, st, g, phi, m, u, x, y, nt);
  return hipGetLastError();
}

hipError_t launch_force(const Geom& g, const double* phi, const double2* eta, const double2* xi, double scale,
                        int accumulate, double* out, int batch, hipStream_t st) {
  const int nt = tiles_of(g.n);
  hipLaunchKernelGGL(k_force, dim3(nt * batch), dim3(kBlock), 0, st, g, phi, eta, xi, scale, accumulate, out, nt);
  return hipGetLastError();
}

hipError_t launch_dot_re(const Geom& g, const double2* a, const double2* b, int batch, double* part,
                         unsigned* counters, double* result, hipStream_t st) {
  const int nt = tiles_of(g.n);
  hipLaunchKernelGGL(k_dot_re, dim3(nt * batch), dim3(kBlock), 0, st, g, a, b, nt, part, counters, result);
  return hipGetLastError();
}

hipError_t launch_phi_to_f32(const double* phi, float* phi32, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_phi_to_f32, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, phi, phi32, n);
  return hipGetLastError();
}

hipError_t launch_cg_iter(const SysDesc* sys, const LaunchList& L, bool single, hipStream_t st) {
  const dim3 grid(L.total_tiles), block(kBlock);
  if (single) {
    hipLaunchKernelGGL((k_cg1<float, float>), grid, block, 0, st, sys, L, (int)S_R32, (int)S_P32, (int)S_U32);
    hipLaunchKernelGGL((k_cg2<float, float>), grid, block, 0, st, sys, L, (int)S_R32, (int)S_P32, (int)S_U32);
  } else {
    hipLaunchKernelGGL((k_cg1<double, double>), grid, block, 0, st, sys, L, (int)S_R, (int)S_P0, (int)S_U);
    hipLaunchKernelGGL((k_cg2<double, double>), grid, block, 0, st, sys, L, (int)S_R, (int)S_P0, (int)S_U);
  }
  return hipGetLastError();
}

hipError_t launch_mdag_slot(const SysDesc* sys, const LaunchList& L, int s_in, bool in_c64, hipStream_t st) {
  const dim3 grid(L.total_tiles), block(kBlock);
  if (in_c64)
    hipLaunchKernelGGL(k_mdag_slot<float2>, grid, block, 0, st, sys, L, s_in);
  else
    hipLaunchKernelGGL(k_mdag_slot<double2>, grid, block, 0, st, sys, L, s_in);
  return hipGetLastError();
}

hipError_t launch_normal2_slot(const SysDesc* sys, const LaunchList& L, int s_in, bool in_c64, int s_b, int s_out,
                               RedMode mode, int red_off, hipStream_t st) {
  const dim3 grid(L.total_tiles), block(kBlock);
  if (in_c64)
    hipLaunchKernelGGL(k_normal2_slot<float2>, grid, block, 0, st, sys, L, s_in, s_b, s_out, (int)mode, red_off);
  else
    hipLaunchKernelGGL(k_normal2_slot<double2>, grid, block, 0, st, sys, L, s_in, s_b, s_out, (int)mode, red_off);
  return hipGetLastError();
}

hipError_t launch_cg_init_zero(const SysDesc* sys, const LaunchList& L, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_init_zero, dim3(L.total_tiles), dim3(kBlock), 0, st, sys, L);
  return hipGetLastError();
}

hipError_t launch_multidot(const SysDesc* sys, const LaunchList& L, int s_w, int s_v0, int cnt, int red_off,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_multidot, dim3(L.total_tiles), dim3(kBlock), 0, st, sys, L, s_w, s_v0, cnt, red_off);
  return hipGetLastError();
}

hipError_t launch_cgs(const SysDesc* sys, const LaunchList& L, int s_w, int s_v0, int cnt, int h_off, int red_off,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_cgs, dim3(L.total_tiles), dim3(kBlock), 0, st, sys, L, s_w, s_v0, cnt, h_off, red_off);
  return hipGetLastError();
}

hipError_t launch_prep_inner(const SysDesc* sys, const LaunchList& L, int s_src, int s_v, hipStream_t st) {
  hipLaunchKernelGGL(k_prep_inner, dim3(L.total_tiles), dim3(kBlock), 0, st, sys, L, s_src, s_v);
  return hipGetLastError();
}

hipError_t launch_xupdate(const SysDesc* sys, const LaunchList& L, int cnt, bool set, hipStream_t st) {
  hipLaunchKernelGGL(k_xupdate, dim3(L.total_tiles), dim3(kBlock), 0, st, sys, L, cnt, set ? 1 : 0);
  return hipGetLastError();
}

}  // namespace hub
