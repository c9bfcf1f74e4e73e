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
//   |r|^2.  Scalars alpha, beta and the convergence test never leave the device;
// * reductions are deterministic and use no atomics: each workgroup stores one
//   partial per tile (wave64 butterfly + fixed LDS combine), and every workgroup of
//   the consuming kernel sums all partials of its system in the same fixed order,
//   so all of them hold bit-identical alpha and beta.  A system's results depend
//   only on its own shape, never on the other systems of the launch.
#include <hip/hip_ext.h>

#include <algorithm>
#include <cstring>
#include <type_traits>

#include "hub_internal.h"

namespace hub {
namespace {

// Loads in flight per thread in the stencil kernels: site pairs of the complex64
// pair path, and sites of the generic path in FP64 and complex64.  With 8 sites
// per thread (tiles of at most 2048 sites) a 102x102x64 system is 768 workgroups,
// resident in one round at the register use these give; more loads per round would
// cost occupancy, fewer (one pair per round: 7 waves per SIMD) made the solve slower.
#ifndef HUB_PAIRS_PER_ROUND
#define HUB_PAIRS_PER_ROUND 2
#endif
#ifndef HUB_SPT64
#define HUB_SPT64 (HUB_SITES_PER_THREAD < 2 ? HUB_SITES_PER_THREAD : 2)
#endif
#ifndef HUB_SPT32
#define HUB_SPT32 (HUB_SITES_PER_THREAD < 2 ? HUB_SITES_PER_THREAD : 2)
#endif
template <typename R> struct Spt;
template <> struct Spt<double> { static constexpr int v = HUB_SPT64; };
template <> struct Spt<float> { static constexpr int v = HUB_SPT32; };

template <typename R> struct V2;
template <> struct V2<double> { using T = double2; };
template <> struct V2<float> { using T = float2; };

// cos x and sin x in FP64 for the public operator kernels (the phase of each site from
// phi): Cody-Waite reduction r = x - q pi/2 with q the integer nearest 2x/pi and pi/2
// split into the nearest double and its remainder (each product inside one FMA, so r is
// exact to an ulp for |q| < 2^20), then the Taylor series of cos r and sin r through
// degree 18 and 17 on |r| <= pi/4 (first omitted terms below 5e-17) and a turn by q
// quarter turns.  Error against e^{ix}: under 2e-16, without the library routine's
// branch for huge arguments.
__device__ __forceinline__ void cis64(double x, double& c, double& s) {
  const double q = rint(x * 0.6366197723675814);
  double r = fma(-q, 1.5707963267948966, x);
  r = fma(-q, 6.123233995736766e-17, r);
  const double r2 = r * r;
  double ps = 2.8114572543455206e-15;         // 1/17!
  ps = fma(ps, r2, -7.647163731819816e-13);   // -1/15!
  ps = fma(ps, r2, 1.6059043836821613e-10);   // 1/13!
  ps = fma(ps, r2, -2.505210838544172e-08);   // -1/11!
  ps = fma(ps, r2, 2.7557319223985893e-06);   // 1/9!
  ps = fma(ps, r2, -0.0001984126984126984);   // -1/7!
  ps = fma(ps, r2, 0.008333333333333333);     // 1/5!
  ps = fma(ps, r2, -0.16666666666666666);     // -1/3!
  const double sr = fma(ps * r2, r, r);
  double pc = 1.5619206968586225e-16;         // 1/18!
  pc = fma(pc, r2, -4.779477332387385e-14);   // -1/16!
  pc = fma(pc, r2, 1.1470745597729725e-11);   // 1/14!
  pc = fma(pc, r2, -2.08767569878681e-09);    // -1/12!
  pc = fma(pc, r2, 2.755731922398589e-07);    // 1/10!
  pc = fma(pc, r2, -2.48015873015873e-05);    // -1/8!
  pc = fma(pc, r2, 0.001388888888888889);     // 1/6!
  pc = fma(pc, r2, -0.041666666666666664);    // -1/4!
  pc = fma(pc, r2, 0.5);                      // 1/2!
  const double cr = fma(-pc, r2, 1.0);
  const int k = (int)q & 3;
  c = (k == 0) ? cr : (k == 1) ? -sr : (k == 2) ? -cr : sr;
  s = (k == 0) ? sr : (k == 1) ? cr : (k == 2) ? -sr : -cr;
}


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

// Views of device vectors in the global address space.  Pointers read from a
// descriptor are generic; accessing them through these views makes the compiler
// emit global_* instead of flat_* memory instructions.
#define HUB_GAS __attribute__((address_space(1)))
typedef double hub_d2v __attribute__((ext_vector_type(2)));
typedef float hub_f2v __attribute__((ext_vector_type(2)));
template <typename C> struct Vec;
template <> struct Vec<double2> {
  HUB_GAS hub_d2v* p;
  __device__ __forceinline__ explicit Vec(const void* q) : p((HUB_GAS hub_d2v*)q) {}
  __device__ __forceinline__ double2 operator[](int k) const {
    const hub_d2v v = p[k];
    double2 r;
    r.x = v.x;
    r.y = v.y;
    return r;
  }
  __device__ __forceinline__ void set(int k, double2 a) const {
    hub_d2v v;
    v.x = a.x;
    v.y = a.y;
    p[k] = v;
  }
};
typedef float hub_f4v __attribute__((ext_vector_type(4)));
// Two consecutive complex64 values (sites k, k+1 with k even: one 16-byte access).
struct C64x2 {
  float2 a, b;
};
template <> struct Vec<float2> {
  HUB_GAS hub_f2v* p;
  __device__ __forceinline__ explicit Vec(const void* q) : p((HUB_GAS hub_f2v*)q) {}
  __device__ __forceinline__ C64x2 pair(int k) const {
    const hub_f4v v = ((HUB_GAS hub_f4v*)p)[k >> 1];
    C64x2 r;
    r.a.x = v.x;
    r.a.y = v.y;
    r.b.x = v.z;
    r.b.y = v.w;
    return r;
  }
  __device__ __forceinline__ void set_pair(int k, C64x2 a) const {
    hub_f4v v;
    v.x = a.a.x;
    v.y = a.a.y;
    v.z = a.b.x;
    v.w = a.b.y;
    ((HUB_GAS hub_f4v*)p)[k >> 1] = v;
  }
  __device__ __forceinline__ float2 operator[](int k) const {
    const hub_f2v v = p[k];
    float2 r;
    r.x = v.x;
    r.y = v.y;
    return r;
  }
  __device__ __forceinline__ void set(int k, float2 a) const {
    hub_f2v v;
    v.x = a.x;
    v.y = a.y;
    p[k] = v;
  }
};
template <typename T> struct Real {
  HUB_GAS T* p;
  __device__ __forceinline__ explicit Real(const void* q) : p((HUB_GAS T*)q) {}
  __device__ __forceinline__ T operator[](int k) const { return p[k]; }
  __device__ __forceinline__ void set(int k, T v) const { p[k] = v; }
  // values at k, k+1 (k even): one 8-byte access for float
  __device__ __forceinline__ hub_f2v pair(int k) const { return ((HUB_GAS hub_f2v*)p)[k >> 1]; }
};

// cos x and sin x in FP32 for the complex64 solver kernels, |x| <= pi in practice (the
// angle is reduced when the solve starts): r = x - q pi/2 with q the integer nearest
// 2x/pi (difference and product in FP64, exact far below FP32 rounding), cos r and
// sin r on |r| <= pi/4 from their Taylor series through degree 10 and 9 (the first
// omitted terms are below 2.5e-9, under half an FP32 ulp), then (cos r, sin r) turned
// by q quarter turns.  Error against e^{ix}: about one FP32 ulp.
__device__ __forceinline__ void cis32(float x, float& c, float& s) {
  const float q = rintf(x * 0.636619772f);
  const float r = (float)fma(-(double)q, 1.5707963267948966, (double)x);
  const float r2 = r * r;
  float ps = fmaf(r2, 2.75573192e-6f, -1.98412698e-4f);  // 1/9!, -1/7!
  ps = fmaf(ps, r2, 8.33333333e-3f);                      // 1/5!
  ps = fmaf(ps, r2, -1.66666667e-1f);                     // -1/3!
  const float sr = fmaf(ps * r2, r, r);
  float pc = fmaf(r2, -2.75573192e-7f, 2.48015873e-5f);  // -1/10!, 1/8!
  pc = fmaf(pc, r2, -1.38888889e-3f);                     // -1/6!
  pc = fmaf(pc, r2, 4.16666667e-2f);                      // 1/4!
  pc = fmaf(pc, r2, -0.5f);
  const float cr = fmaf(pc, r2, 1.0f);
  const int k = (int)q & 3;
  c = (k == 0) ? cr : (k == 1) ? -sr : (k == 2) ? -cr : sr;
  s = (k == 0) ? sr : (k == 1) ? cr : (k == 2) ? -sr : -cr;
}

// The phase e^{i phi} a stencil needs, from one of three sources:
//  * AnglePhi - phi itself (FP64); cos and sin from cis64 per site (the public
//               operator kernels, whose input is phi);
//  * PhasePhi - (cos phi, sin phi) precomputed once per solve (the FP64 solver
//               kernels: a 16-byte load replaces a sincos per site);
//  * Angle32  - phi reduced to [-pi, pi] and rounded to float once per solve, cos and
//               sin from cis32 (the complex64 solver kernels: a 4-byte load and a few
//               FMAs, against 8 bytes for a precomputed complex64 phase).
// load(k) returns the raw value of site k, cs() turns it into (cos, sin); load2 / cs2
// do the same for the two sites k, k+1 (k even) of the complex64 pair path.
template <typename R> struct AnglePhi;
template <> struct AnglePhi<double> {
  Real<double> a;
  using Raw = double;
  __device__ __forceinline__ explicit AnglePhi(const void* q) : a(q) {}
  __device__ __forceinline__ Raw load(int k) const { return a[k]; }
  __device__ __forceinline__ void cs(Raw v, double& c, double& s) const { cis64(v, c, s); }
};
struct Angle32 {
  Real<float> a;
  using Raw = float;
  using Raw2 = hub_f2v;
  __device__ __forceinline__ explicit Angle32(const void* q) : a(q) {}
  __device__ __forceinline__ Raw load(int k) const { return a[k]; }
  __device__ __forceinline__ void cs(Raw v, float& c, float& s) const { cis32(v, c, s); }
  __device__ __forceinline__ Raw2 load2(int k) const { return a.pair(k); }
  __device__ __forceinline__ void cs2(Raw2 v, int h, float& c, float& s) const { cis32(h ? v.y : v.x, c, s); }
};
template <typename R> struct PhasePhi {
  using C = typename V2<R>::T;
  Vec<C> p;
  using Raw = C;
  using Raw2 = C64x2;
  __device__ __forceinline__ explicit PhasePhi(const void* q) : p(q) {}
  __device__ __forceinline__ Raw load(int k) const { return p[k]; }
  __device__ __forceinline__ void cs(Raw v, R& c, R& s) const {
    c = v.x;
    s = v.y;
  }
  __device__ __forceinline__ Raw2 load2(int k) const { return p.pair(k); }
  __device__ __forceinline__ void cs2(Raw2 v, int h, float& c, float& s) const {
    c = h ? v.b.x : v.a.x;
    s = h ? v.b.y : v.a.y;
  }
};

// The stencil of M (DAG = false) or M^dagger (DAG = true) at site n (eq. (ferm_op) and its
// conjugate transpose):
//   M,  A row: -x(n) + s (e^{ i phi(n)}  - m) x(t-1) - kappa sum_bonds x_B
//   M,  B row: +x(n) - s (e^{-i phi(n)}  - m) x(t+1) - kappa sum_bonds x_A
//   M+, A row: -x(n) + s (e^{-i phi(tn)} - m) x(t+1) - kappa sum_bonds x_B
//   M+, B row: +x(n) - s (e^{ i phi(tn)} - m) x(t-1) - kappa sum_bonds x_A
// with s = -1 on a hop across the antiperiodic temporal boundary.
//
// Index part of the stencil at site n: own site, temporal
// neighbour, three bonds, the phi index and the row's signs.
struct SiteIdx {
  int n, tn, h0, h1, h2, pn;
  bool isA;
  bool wrap;
};

// The same from the coordinates of site n: cell (i, j) and plane q2 = 2 t + s.
template <bool DAG>
__device__ __forceinline__ SiteIdx site_index_at(const Geom& g, int n, int i, int j, uint32_t q2) {
  SiteIdx s;
  s.isA = (q2 & 1u) == 0;
  const int t = (int)(q2 >> 1);
  const int P2 = 2 * g.P;
  if (s.isA == DAG) {
    s.wrap = t == g.Nt - 1;
    s.tn = s.wrap ? n - (g.Nt - 1) * P2 : n + P2;
  } else {
    s.wrap = t == 0;
    s.tn = s.wrap ? n + (g.Nt - 1) * P2 : n - P2;
  }
  if (s.isA) {
    const int b = n + g.P;
    s.h0 = b;
    s.h1 = (i > 0) ? b - g.L2 : b + (g.L1 - 1) * g.L2;
    s.h2 = (j > 0) ? b - 1 : b + g.L2 - 1;
  } else {
    const int a = n - g.P;
    s.h0 = a;
    s.h1 = (i < g.L1 - 1) ? a + g.L2 : a - (g.L1 - 1) * g.L2;
    s.h2 = (j < g.L2 - 1) ? a + 1 : a - (g.L2 - 1);
  }
  s.n = n;
  s.pn = DAG ? s.tn : n;
  return s;
}

template <bool DAG>
__device__ __forceinline__ SiteIdx site_index(const Geom& g, int n) {
  const uint32_t q1 = fdiv((uint32_t)n, g.dL2);
  const int j = n - (int)q1 * g.L2;
  const uint32_t q2 = fdiv(q1, g.dL1);
  const int i = (int)q1 - (int)q2 * g.L1;
  return site_index_at<DAG>(g, n, i, j, q2);
}

template <typename R, bool DAG, typename C>
__device__ __forceinline__ C stencil_combine(const Geom& g, const SiteIdx& st, R c, R s, C xs, C xt, C x0, C x1,
                                             C x2) {
  const R sgn = st.wrap ? R(-1) : R(1);
  const R es = (st.isA != DAG) ? s : -s;
  const R cr = sgn * (c - (R)g.ms), ci = sgn * es;
  const R tr = cr * xt.x - ci * xt.y, ti = cr * xt.y + ci * xt.x;
  const R sig = st.isA ? R(-1) : R(1);
  const R kap = (R)g.kappa;
  C y;
  y.x = sig * (xs.x - tr) - kap * (x0.x + x1.x + x2.x);
  y.y = sig * (xs.y - ti) - kap * (x0.y + x1.y + x2.y);
  return y;
}

// Apply the stencil to the kSitesPerThread sites of this thread in a tile, SPT
// sites at a time: all index arithmetic first, then every load of the SPT sites
// (raw stencil inputs `ld`, phi and the epilogue's own operands `pre`), then, in
// the first round only, `mid()` (which may compute scalars from partial sums and
// returns false to skip the rest), then `cook(raw)` turns raw loads into stencil
// inputs, the arithmetic, and `post(n, y, self, pre_value)`.  Issuing the loads
// of several sites before the first wait keeps enough bytes in flight to cover
// HBM latency, and the partial-sum prologue of `mid` overlaps those loads.  The
// thread's sites are base + m*kBlock below `end` (the end of its tile); lanes past
// it load a valid site and skip `post`.
template <typename R, bool DAG, int SPT, int TOTAL = kSitesPerThread, typename Phi, typename Load, typename Cook,
          typename Pre, typename Mid, typename Post>
__device__ __forceinline__ void stencil_sites(const Geom& g, const Phi& phi, int base, int end, Load ld, Cook cook,
                                              Pre pre, Mid mid, Post post) {
  using C = typename V2<R>::T;
  using RW = decltype(ld(0));
  using PV = decltype(pre(0));
  static_assert(TOTAL % SPT == 0, "SPT must divide TOTAL");
#pragma unroll
  for (int r0 = 0; r0 < TOTAL; r0 += SPT) {
    SiteIdx st[SPT];
    bool ok[SPT];
#pragma unroll
    for (int m = 0; m < SPT; ++m) {
      int n = base + (r0 + m) * kBlock;
      ok[m] = n < end;
      n = ok[m] ? n : end - 1;
      st[m] = site_index<DAG>(g, n);
    }
    RW xs[SPT], xt[SPT], x0[SPT], x1[SPT], x2[SPT];
    typename Phi::Raw ph[SPT];
    PV pv[SPT];
#pragma unroll
    for (int m = 0; m < SPT; ++m) {
      xs[m] = ld(st[m].n);
      xt[m] = ld(st[m].tn);
      x0[m] = ld(st[m].h0);
      x1[m] = ld(st[m].h1);
      x2[m] = ld(st[m].h2);
      ph[m] = phi.load(st[m].pn);
      pv[m] = pre(st[m].n);
    }
    if (r0 == 0 && !mid()) return;
#pragma unroll
    for (int m = 0; m < SPT; ++m) {
      const C s0 = cook(xs[m]);
      R c, s;
      phi.cs(ph[m], c, s);
      const C y = stencil_combine<R, DAG>(g, st[m], c, s, s0, cook(xt[m]), cook(x0[m]), cook(x1[m]),
                                          cook(x2[m]));
      if (ok[m]) post(st[m].n, y, s0, pv[m]);
    }
  }
}

struct NoMid {
  __device__ __forceinline__ bool operator()() const { return true; }
};
struct Same {
  template <typename T>
  __device__ __forceinline__ T operator()(T v) const {
    return v;
  }
};

struct NoPre {
  int dummy;
};

// ---------------------------------------------------------------------------
// Complex64 stencil on site pairs (j, j+1), j even, for lattices with even L2.
// A pair never straddles a row, so the own values, the temporal neighbours, the
// sublattice partners and the i-neighbour row are 16-byte loads of two sites; of
// the j-bonds one is the partner load's other half and one is an extra 8-byte
// load.  This halves the memory instructions per site of the complex64 kernels.
// ---------------------------------------------------------------------------
struct PairIdx {
  int n, tn, h0, h1, hx;
  bool isA, wrap;
};

// Index part of the stencil on the pair (n, n + 1), n even, from the coordinates of
// site n: cell (i, j) and plane q2 = 2 t + s.
template <bool DAG>
__device__ __forceinline__ PairIdx pair_index_at(const Geom& g, int n, int i, int j, uint32_t q2) {
  PairIdx s;
  s.isA = (q2 & 1u) == 0;
  const int t = (int)(q2 >> 1);
  const int P2 = 2 * g.P;
  if (s.isA == DAG) {
    s.wrap = t == g.Nt - 1;
    s.tn = s.wrap ? n - (g.Nt - 1) * P2 : n + P2;
  } else {
    s.wrap = t == 0;
    s.tn = s.wrap ? n + (g.Nt - 1) * P2 : n - P2;
  }
  if (s.isA) {
    const int b = n + g.P;
    s.h0 = b;
    s.h1 = (i > 0) ? b - g.L2 : b + (g.L1 - 1) * g.L2;
    s.hx = (j > 0) ? b - 1 : b + g.L2 - 1;  // B(i, j-1)
  } else {
    const int a = n - g.P;
    s.h0 = a;
    s.h1 = (i < g.L1 - 1) ? a + g.L2 : a - (g.L1 - 1) * g.L2;
    s.hx = (j + 2 < g.L2) ? a + 2 : a + 2 - g.L2;  // A(i, j+2)
  }
  s.n = n;
  return s;
}

template <bool DAG>
__device__ __forceinline__ PairIdx pair_index(const Geom& g, int n) {
  const uint32_t q1 = fdiv((uint32_t)n, g.dL2);
  const int j = n - (int)q1 * g.L2;
  const uint32_t q2 = fdiv(q1, g.dL1);
  const int i = (int)q1 - (int)q2 * g.L1;
  return pair_index_at<DAG>(g, n, i, j, q2);
}

// The stencil on one site pair: own values xs, temporal neighbours xt, the partner
// pair x0, the i-neighbour pair x1 and the extra j-neighbour xe; csf(h, c, s) gives the
// phase (cos, sin) of row h of the pair, evaluated as the row is reached.
template <bool DAG, typename CsF>
__device__ __forceinline__ C64x2 pair_stencil(const Geom& g, const PairIdx& sm, CsF csf, C64x2 xs, C64x2 xt,
                                              C64x2 x0, C64x2 x1, float2 xe) {
  // bond sums of the two sites
  float2 b0, b1;
  if (sm.isA) {
    b0.x = x0.a.x + x1.a.x + xe.x;
    b0.y = x0.a.y + x1.a.y + xe.y;
    b1.x = x0.b.x + x1.b.x + x0.a.x;
    b1.y = x0.b.y + x1.b.y + x0.a.y;
  } else {
    b0.x = x0.a.x + x1.a.x + x0.b.x;
    b0.y = x0.a.y + x1.a.y + x0.b.y;
    b1.x = x0.b.x + x1.b.x + xe.x;
    b1.y = x0.b.y + x1.b.y + xe.y;
  }
  const float sgn = sm.wrap ? -1.0f : 1.0f;
  const float sig = sm.isA ? -1.0f : 1.0f;
  const float kap = (float)g.kappa, mst = (float)g.ms;
  const bool plus = (sm.isA != DAG);
  C64x2 y;
  {
    float c0, s0;
    csf(0, c0, s0);
    const float es = plus ? s0 : -s0;
    const float cr = sgn * (c0 - mst), ci = sgn * es;
    const float tr = cr * xt.a.x - ci * xt.a.y, ti = cr * xt.a.y + ci * xt.a.x;
    y.a.x = sig * (xs.a.x - tr) - kap * b0.x;
    y.a.y = sig * (xs.a.y - ti) - kap * b0.y;
  }
  {
    float c1, s1;
    csf(1, c1, s1);
    const float es = plus ? s1 : -s1;
    const float cr = sgn * (c1 - mst), ci = sgn * es;
    const float tr = cr * xt.b.x - ci * xt.b.y, ti = cr * xt.b.y + ci * xt.b.x;
    y.b.x = sig * (xs.b.x - tr) - kap * b1.x;
    y.b.y = sig * (xs.b.y - ti) - kap * b1.y;
  }
  return y;
}

// Apply M (DAG = false) or M^dagger to the TOTAL/2 site pairs of this thread in the
// tile of sites [lo, end) (lo even, at most kBlock * TOTAL sites): the pairs starting
// at lo + 2*(threadIdx.x + m*kBlock) below end.  ld2(k) loads the raw
// input at k, k+1 and ld1(k) at k; after `mid()` (see stencil_sites), cook2 / cook1
// turn them into C64x2 / float2 inputs; post(n, y, self, pre) per pair.
template <bool DAG, int TOTAL = kSitesPerThread, typename Phi, typename Ld2, typename Ld1, typename Cook2,
          typename Cook1, typename Pre, typename Mid, typename Post>
__device__ __forceinline__ void stencil_pairs(const Geom& g, const Phi& phi, int lo, int end, Ld2 ld2, Ld1 ld1,
                                              Cook2 cook2, Cook1 cook1, Pre pre, Mid mid, Post post) {
  using PV = decltype(pre(0));
  using R2 = decltype(ld2(0));
  using R1 = decltype(ld1(0));
  constexpr int NPT = TOTAL / 2;  // pairs per thread
  constexpr int NP = HUB_PAIRS_PER_ROUND < NPT ? HUB_PAIRS_PER_ROUND : NPT;  // pairs in flight per round
  static_assert(NPT % NP == 0, "rounds must divide the pairs");
#pragma unroll
  for (int q0 = 0; q0 < NPT; q0 += NP) {
  PairIdx st[NP];
  bool ok[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    int n = lo + 2 * (threadIdx.x + (q0 + m) * kBlock);
    ok[m] = n < end;
    n = ok[m] ? n : end - 2;
    st[m] = pair_index<DAG>(g, n);
  }
  R2 rs[NP], rt[NP], r0[NP], r1[NP];
  R1 re[NP];
  typename Phi::Raw2 ph[NP];
  PV pv[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    rs[m] = ld2(st[m].n);
    rt[m] = ld2(st[m].tn);
    r0[m] = ld2(st[m].h0);
    r1[m] = ld2(st[m].h1);
    re[m] = ld1(st[m].hx);
    ph[m] = phi.load2(DAG ? st[m].tn : st[m].n);
    pv[m] = pre(st[m].n);
  }
  if (q0 == 0 && !mid()) return;
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    const PairIdx& sm = st[m];
    const C64x2 xs = cook2(rs[m]), xt = cook2(rt[m]), x0 = cook2(r0[m]), x1 = cook2(r1[m]);
    const float2 xe = cook1(re[m]);
    // the arithmetic of pair_stencil, written out here: through the helper the compiler
    // schedules this loop with 10 more registers per thread
    float2 b0, b1;
    if (sm.isA) {
      b0.x = x0.a.x + x1.a.x + xe.x;
      b0.y = x0.a.y + x1.a.y + xe.y;
      b1.x = x0.b.x + x1.b.x + x0.a.x;
      b1.y = x0.b.y + x1.b.y + x0.a.y;
    } else {
      b0.x = x0.a.x + x1.a.x + x0.b.x;
      b0.y = x0.a.y + x1.a.y + x0.b.y;
      b1.x = x0.b.x + x1.b.x + xe.x;
      b1.y = x0.b.y + x1.b.y + xe.y;
    }
    const float sgn = sm.wrap ? -1.0f : 1.0f;
    const float sig = sm.isA ? -1.0f : 1.0f;
    const float kap = (float)g.kappa, mst = (float)g.ms;
    const bool plus = (sm.isA != DAG);
    C64x2 y;
    {
      float c, s;
      phi.cs2(ph[m], 0, c, s);
      const float es = plus ? s : -s;
      const float cr = sgn * (c - mst), ci = sgn * es;
      const float tr = cr * xt.a.x - ci * xt.a.y, ti = cr * xt.a.y + ci * xt.a.x;
      y.a.x = sig * (xs.a.x - tr) - kap * b0.x;
      y.a.y = sig * (xs.a.y - ti) - kap * b0.y;
    }
    {
      float c, s;
      phi.cs2(ph[m], 1, c, s);
      const float es = plus ? s : -s;
      const float cr = sgn * (c - mst), ci = sgn * es;
      const float tr = cr * xt.b.x - ci * xt.b.y, ti = cr * xt.b.y + ci * xt.b.x;
      y.b.x = sig * (xs.b.x - tr) - kap * b1.x;
      y.b.y = sig * (xs.b.y - ti) - kap * b1.y;
    }
    if (ok[m]) post(sm.n, y, xs, pv[m]);
  }
  }
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

// Sum of `cnt` partials spaced `stride` apart, fixed order, same value in every thread.
__device__ __forceinline__ double sum_partials(const double* part, int cnt, int stride) {
  const Real<double> p(part);
  double acc = 0.0;
  for (int k = threadIdx.x; k < cnt; k += kBlock) acc += p[k * stride];
  return block_sum(acc);
}

template <typename LL>
__device__ __forceinline__ int find_sys(const LL& L, int lt) {
  int lo = 0, hi = L.nsys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (L.tile_begin[mid] <= lt) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The phase source of the solver kernels in precision R.
template <typename R> struct SolverPhase;
template <> struct SolverPhase<double> { using T = PhasePhi<double>; };
template <> struct SolverPhase<float> { using T = Angle32; };
template <typename R> __device__ __forceinline__ typename SolverPhase<R>::T phase_of(const SysDesc* d);
template <> __device__ __forceinline__ PhasePhi<double> phase_of<double>(const SysDesc* d) {
  return PhasePhi<double>(d->ph64);
}
template <> __device__ __forceinline__ Angle32 phase_of<float>(const SysDesc* d) { return Angle32(d->ph32); }

__device__ __forceinline__ int load_active(Scal* sc) {
  return __hip_atomic_load(&sc->active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_active(Scal* sc, int v) {
  __hip_atomic_store(&sc->active, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Public operator kernels (shared phi, batch of vectors, no descriptors).  They
// have no reduction partials, so they use smaller tiles (two sites per thread,
// both loaded together): more waves in flight than the CG kernels' tiles.  A
// workgroup applies the operator to a group of `per` consecutive vectors of the
// batch: the site indices, phi and its phase are loaded and evaluated once per site
// for the whole group (the launcher makes the group the whole batch whenever the
// lattice alone gives enough workgroups).
// ---------------------------------------------------------------------------
constexpr int kPubSites = 2;
constexpr int kPubTile = kBlock * kPubSites;

// Store of an operator result.  NT = true: a non-temporal store, for outputs handed
// back to the caller (the result is not read again by this launch or the next one;
// at 102x102x64 the public FP64 apply takes 8.1-8.6 us instead of 10.2 us with its
// working set in the infinity cache and 13.7-14.2 us instead of 15.3 us with buffers
// rotated past it).  NT = false: a plain store, for results a following kernel of the
// library reads at once (xi for the force, the first pass of the normal operator),
// which a non-temporal store would send past the infinity cache.
template <bool NT>
__device__ __forceinline__ void store_out(double2* p, double2 v) {
  if constexpr (NT) {
    hub_d2v w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, (hub_d2v*)p);
  } else {
    *p = v;
  }
}

// One vector per workgroup: all loads of a round in flight together, then the phase.
template <bool DAG, bool NT>
__global__ __launch_bounds__(kBlock) void k_apply(Geom g, const double* __restrict__ phi,
                                                  const double2* __restrict__ x, double2* __restrict__ y,
                                                  int ntiles) {
  const int l = xcd_remap(blockIdx.x, gridDim.x);
  const int b = l / ntiles, tile = l - b * ntiles;
  const double2* __restrict__ xb = x + (size_t)b * g.n;
  double2* __restrict__ yb = y + (size_t)b * g.n;
  const int base = tile * kPubTile + threadIdx.x;
  auto ld = [=](int k) { return xb[k]; };
  auto pre = [](int) { return NoPre{}; };
  auto post = [=](int n, double2 v, double2, NoPre) { store_out<NT>(yb + n, v); };
  stencil_sites<double, DAG, kPubSites, kPubSites>(g, AnglePhi<double>(phi), base, g.n, ld, Same{}, pre, NoMid{},
                                                   post);
}

// A group of `per` vectors per workgroup (separate kernel, so that the one-vector
// kernel keeps its register budget).
template <bool DAG, bool NT>
__global__ __launch_bounds__(kBlock) void k_apply_grp(Geom g, const double* __restrict__ phi,
                                                      const double2* __restrict__ x, double2* __restrict__ y,
                                                      int ntiles, int per, int batch) {
  const int l = xcd_remap(blockIdx.x, gridDim.x);
  const int grp = l / ntiles, tile = l - grp * ntiles;
  const int b0 = grp * per, b1 = min(batch, b0 + per);
  const int base = tile * kPubTile + threadIdx.x;
  SiteIdx st[kPubSites];
  bool ok[kPubSites];
  double ph[kPubSites], c[kPubSites], s[kPubSites];
#pragma unroll
  for (int m = 0; m < kPubSites; ++m) {
    int n = base + m * kBlock;
    ok[m] = n < g.n;
    n = ok[m] ? n : g.n - 1;
    st[m] = site_index<DAG>(g, n);
    ph[m] = phi[st[m].pn];
  }
  for (int b = b0; b < b1; ++b) {
    const double2* __restrict__ xb = x + (size_t)b * g.n;
    double2* __restrict__ yb = y + (size_t)b * g.n;
    double2 xs[kPubSites], xt[kPubSites], x0[kPubSites], x1[kPubSites], x2[kPubSites];
#pragma unroll
    for (int m = 0; m < kPubSites; ++m) {
      xs[m] = xb[st[m].n];
      xt[m] = xb[st[m].tn];
      x0[m] = xb[st[m].h0];
      x1[m] = xb[st[m].h1];
      x2[m] = xb[st[m].h2];
    }
    if (b == b0) {
#pragma unroll
      for (int m = 0; m < kPubSites; ++m) cis64(ph[m], c[m], s[m]);
    }
#pragma unroll
    for (int m = 0; m < kPubSites; ++m) {
      const double2 v = stencil_combine<double, DAG>(g, st[m], c[m], s[m], xs[m], xt[m], x0[m], x1[m], x2[m]);
      if (ok[m]) store_out<NT>(yb + st[m].n, v);
    }
  }
}

struct Mu2Arr { double v[kMaxSys]; };

// y_b = M u_b + mu2_b x_b: the second pass of the public normal operator (u = M^dagger x),
// one vector per workgroup.
__global__ __launch_bounds__(kBlock) void k_normal2_pub(Geom g, const double* __restrict__ phi, Mu2Arr mu2,
                                                        const double2* __restrict__ u,
                                                        const double2* __restrict__ x, double2* __restrict__ y,
                                                        int ntiles) {
  const int l = xcd_remap(blockIdx.x, gridDim.x);
  const int b = l / ntiles, tile = l - b * ntiles;
  const size_t off = (size_t)b * g.n;
  const double m2 = mu2.v[b];
  const int base = tile * kPubTile + threadIdx.x;
  auto ld = [=](int k) { return u[off + k]; };
  auto pre = [=](int n) { return x[off + n]; };
  auto post = [=](int n, double2 q, double2, double2 xv) {
    q.x += m2 * xv.x;
    q.y += m2 * xv.y;
    y[off + n] = q;
  };
  stencil_sites<double, false, kPubSites, kPubSites>(g, AnglePhi<double>(phi), base, g.n, ld, Same{}, pre, NoMid{},
                                                     post);
}

// The same for a group of `per` vectors per workgroup.
__global__ __launch_bounds__(kBlock) void k_normal2_grp(Geom g, const double* __restrict__ phi, Mu2Arr mu2,
                                                        const double2* __restrict__ u,
                                                        const double2* __restrict__ x, double2* __restrict__ y,
                                                        int ntiles, int per, int batch) {
  const int l = xcd_remap(blockIdx.x, gridDim.x);
  const int grp = l / ntiles, tile = l - grp * ntiles;
  const int b0 = grp * per, b1 = min(batch, b0 + per);
  const int base = tile * kPubTile + threadIdx.x;
  SiteIdx st[kPubSites];
  bool ok[kPubSites];
  double ph[kPubSites], c[kPubSites], s[kPubSites];
#pragma unroll
  for (int m = 0; m < kPubSites; ++m) {
    int n = base + m * kBlock;
    ok[m] = n < g.n;
    n = ok[m] ? n : g.n - 1;
    st[m] = site_index<false>(g, n);
    ph[m] = phi[st[m].pn];
  }
  for (int b = b0; b < b1; ++b) {
    const size_t off = (size_t)b * g.n;
    const double m2 = mu2.v[b];
    double2 us[kPubSites], ut[kPubSites], u0[kPubSites], u1[kPubSites], u2[kPubSites], xv[kPubSites];
#pragma unroll
    for (int m = 0; m < kPubSites; ++m) {
      us[m] = u[off + st[m].n];
      ut[m] = u[off + st[m].tn];
      u0[m] = u[off + st[m].h0];
      u1[m] = u[off + st[m].h1];
      u2[m] = u[off + st[m].h2];
      xv[m] = x[off + st[m].n];
    }
    if (b == b0) {
#pragma unroll
      for (int m = 0; m < kPubSites; ++m) cis64(ph[m], c[m], s[m]);
    }
#pragma unroll
    for (int m = 0; m < kPubSites; ++m) {
      double2 q = stencil_combine<double, false>(g, st[m], c[m], s[m], us[m], ut[m], u0[m], u1[m], u2[m]);
      q.x += m2 * xv[m].x;
      q.y += m2 * xv[m].y;
      if (ok[m]) y[off + st[m].n] = q;
    }
  }
}

// Vectors per workgroup of the public batched kernels: the whole batch when the
// lattice alone gives about 1024 workgroups or more, else fewer so that the launch
// still has that many.
static int pub_group(int ntiles, int batch) {
  const long want = 1024;
  const long per = (long)ntiles * batch / want;
  return (int)std::max<long>(1, std::min<long>(batch, per));
}

// dS/dphi at every site: A: 2 Im[conj(eta(t)) s e^{i phi} z(t-1)],
//                        B: 2 Im[conj(eta(t)) s e^{-i phi} z(t+1)],
// with z = xi, or z = xi - sub for the ratio terms of the Hasenbusch split
// (eq. (f_chi_i)); the derivative of M does not depend on the staggered mass.
__global__ __launch_bounds__(kBlock) void k_force(Geom g, const double* __restrict__ phi,
                                                  const double2* __restrict__ eta,
                                                  const double2* __restrict__ xi,
                                                  const double2* __restrict__ sub, double scale, int accumulate,
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
      cis64(phi[n], c, s);
      if (!isA) s = -s;
      const double2 e = eta[off + n];
      double2 z = xi[off + tn];
      if (sub) {
        const double2 v = sub[off + tn];
        z.x -= v.x;
        z.y -= v.y;
      }
      // w = sgn (c + i s) z ; F = 2 Im(conj(e) w)
      const double wr = sgn * (c * z.x - s * z.y), wi = sgn * (c * z.y + s * z.x);
      const double F = 2.0 * (e.x * wi - e.y * wr);
      double* o = out + off + n;
      *o = accumulate ? *o + scale * F : scale * F;
    }
  }
}

// The same for a group of `per` vectors per workgroup: the temporal neighbour and
// the phase of each site are evaluated once for the group.
__global__ __launch_bounds__(kBlock) void k_force_grp(Geom g, const double* __restrict__ phi,
                                                      const double2* __restrict__ eta,
                                                      const double2* __restrict__ xi,
                                                      const double2* __restrict__ sub, double scale, int accumulate,
                                                      double* __restrict__ out, int ntiles, int per, int batch) {
  const int l = xcd_remap(blockIdx.x, gridDim.x);
  const int grp = l / ntiles, tile = l - grp * ntiles;
  const int b0 = grp * per, b1 = min(batch, b0 + per);
  const int base = tile * kTile + threadIdx.x;
  const int P2 = 2 * g.P;
  // per site: the temporal neighbour and s e^{+-i phi}, shared by the vectors of the group
  int tn[kSitesPerThread];
  double ec[kSitesPerThread], es[kSitesPerThread];
#pragma unroll
  for (int m = 0; m < kSitesPerThread; ++m) {
    const int n = min(base + m * kBlock, g.n - 1);
    const uint32_t q2 = fdiv(fdiv((uint32_t)n, g.dL2), g.dL1);
    const bool isA = (q2 & 1u) == 0;
    const int t = (int)(q2 >> 1);
    double sgn;
    if (isA) {
      const bool wrap = t == 0;
      tn[m] = wrap ? n + (g.Nt - 1) * P2 : n - P2;
      sgn = wrap ? -1.0 : 1.0;
    } else {
      const bool wrap = t == g.Nt - 1;
      tn[m] = wrap ? n - (g.Nt - 1) * P2 : n + P2;
      sgn = wrap ? -1.0 : 1.0;
    }
    double c, s;
    cis64(phi[n], c, s);
    ec[m] = sgn * c;
    es[m] = sgn * (isA ? s : -s);
  }
  for (int b = b0; b < b1; ++b) {
    const size_t off = (size_t)b * g.n;
#pragma unroll
    for (int m = 0; m < kSitesPerThread; ++m) {
      const int n = base + m * kBlock;
      if (n < g.n) {
        const double2 e = eta[off + n];
        double2 z = xi[off + tn[m]];
        if (sub) {
          const double2 v = sub[off + tn[m]];
          z.x -= v.x;
          z.y -= v.y;
        }
        // w = s e^{+-i phi} z ; F = 2 Im(conj(e) w)
        const double wr = ec[m] * z.x - es[m] * z.y, wi = ec[m] * z.y + es[m] * z.x;
        const double F = 2.0 * (e.x * wi - e.y * wr);
        double* o = out + off + n;
        *o = accumulate ? *o + scale * F : scale * F;
      }
    }
  }
}

// Sum over the vectors of a batch: out (+)= sum_b scale_b F_b with F_b the force of
// k_force.  phi, its phase and the temporal neighbour are evaluated once per site; per
// site and vector only eta and xi (at the neighbour) are read, and out is written once.
__global__ __launch_bounds__(kBlock) void k_force_sum(Geom g, const double* __restrict__ phi,
                                                      const double2* __restrict__ eta,
                                                      const double2* __restrict__ xi, Mu2Arr scale,
                                                      int accumulate, double* __restrict__ out, int batch) {
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int base = tile * kTile + threadIdx.x;
  const int P2 = 2 * g.P;
#pragma unroll 2
  for (int m = 0; m < kSitesPerThread; ++m) {
    const int n = base + m * kBlock;
    if (n >= g.n) break;
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
    cis64(phi[n], c, s);
    const double ec = sgn * c, es = sgn * (isA ? s : -s);
    double F = 0.0;
    for (int b = 0; b < batch; ++b) {
      const size_t off = (size_t)b * g.n;
      const double2 e = eta[off + n];
      const double2 z = xi[off + tn];
      // w = s e^{+-i phi} z ; F_b = 2 Im(conj(e) w)
      const double wr = ec * z.x - es * z.y, wi = ec * z.y + es * z.x;
      F = fma(scale.v[b], 2.0 * (e.x * wi - e.y * wr), F);
    }
    out[n] = accumulate ? out[n] + F : F;
  }
}

// Measurement only: the bytes of one FP64 apply (x and phi read, y written per site)
// with no stencil and no phase, two sites per thread, the apply's grid and workgroup
// order.  NTL: non-temporal loads; NTS: non-temporal stores.
template <bool NTL, bool NTS>
__global__ __launch_bounds__(kBlock) void k_stream_bytes(const double* __restrict__ phi,
                                                         const double2* __restrict__ x, double2* __restrict__ y,
                                                         int n) {
  const int l = xcd_remap(blockIdx.x, gridDim.x);
  const int base = l * kPubTile + threadIdx.x;
  double2 v[kPubSites];
  double p[kPubSites];
#pragma unroll
  for (int m = 0; m < kPubSites; ++m) {
    const int k = min(base + m * kBlock, n - 1);
    if constexpr (NTL) {
      const hub_d2v w = __builtin_nontemporal_load((const hub_d2v*)(x + k));
      v[m].x = w.x;
      v[m].y = w.y;
      p[m] = __builtin_nontemporal_load(phi + k);
    } else {
      v[m] = x[k];
      p[m] = phi[k];
    }
  }
#pragma unroll
  for (int m = 0; m < kPubSites; ++m) {
    const int k = base + m * kBlock;
    double2 o;
    o.x = v[m].x * p[m];
    o.y = v[m].y + p[m];
    if (k < n) store_out<NTS>(y + k, o);
  }
}

// Per-tile partials of Re sum conj(a_b) b_b.
__global__ __launch_bounds__(kBlock) void k_dot_re(Geom g, const double2* __restrict__ a,
                                                   const double2* __restrict__ bb, int ntiles,
                                                   double* __restrict__ part) {
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
  const double tot = block_sum(acc);
  if (threadIdx.x == 0) part[(size_t)b * ntiles + tile] = tot;
}

// result[b] = fixed-order sum of the partials of system b (one workgroup each).
__global__ __launch_bounds__(kBlock) void k_dot_finish(const double* __restrict__ part, int ntiles,
                                                       double* __restrict__ result) {
  const double s = sum_partials(part + (size_t)blockIdx.x * ntiles, ntiles, 1);
  if (threadIdx.x == 0) result[blockIdx.x] = s;
}

// (cos phi, sin phi) per site in FP64 and, when p32 is given, phi - 2 pi k (k the
// integer nearest phi / 2 pi, in FP64) rounded to float.
__global__ __launch_bounds__(kBlock) void k_phase(const double* __restrict__ phi, double2* __restrict__ p64,
                                                  float* __restrict__ p32, float2* __restrict__ cs32, int n) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double a = phi[i];
  double c, s;
  sincos(a, &s, &c);
  double2 v;
  v.x = c;
  v.y = s;
  p64[i] = v;
  const float a32 = (float)fma(-rint(a * 0.15915494309189535), 6.283185307179586, a);
  if (p32) p32[i] = a32;
  if (cs32) {
    // the complex64 kernels' phase of that angle, as they would evaluate it
    float2 e;
    cis32(a32, e.x, e.y);
    cs32[i] = e;
  }
}

// Molecular dynamics (Sec. 5.2): phi += eps pi (T_pi), and the momentum kick
// pi -= G + cg phi, where G holds the summed pseudofermion force contributions
// sum_k eps_k dS_k/dphi and cg = eps/U~ is the gauge force's share.
__global__ __launch_bounds__(kBlock) void k_md_drift(double* __restrict__ phi, const double* __restrict__ pi,
                                                     double eps, int n) {
  const int i = xcd_remap(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i < n) phi[i] += eps * pi[i];
}

__global__ __launch_bounds__(kBlock) void k_md_kick(double* __restrict__ pi, const double* __restrict__ phi,
                                                    const double* __restrict__ G, double cg, int n) {
  const int i = xcd_remap(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i < n) pi[i] -= (G ? G[i] : 0.0) + cg * phi[i];
}

// ---------------------------------------------------------------------------
// Batched solver kernels (descriptor + launch list).
// ---------------------------------------------------------------------------
// Sites [lo, hi) of solver tile `tile` (block tile % nb of segment tile / nb).
struct TileRange {
  int lo, hi;
};
__device__ __forceinline__ TileRange tile_range(int tile, int nb, int bsz, int seg) {
  const int sg = tile / nb;
  TileRange r;
  r.lo = sg * seg + (tile - sg * nb) * bsz;
  r.hi = min(r.lo + bsz, (sg + 1) * seg);
  return r;
}

// Prologue of the batched solver kernels: the system and tile of this workgroup.
// The tile holds the sites [t_lo, t_hi) (block tile % tnb of segment tile / tnb, at
// most TILE sites: every kernel of a system uses the tile size of its class); the
// thread's sites are base + m*kBlock below t_hi.
#define HUB_PROLOGUE_T(TILE)                                            \
  const int lt = xcd_remap(blockIdx.x, gridDim.x);                      \
  const int kk = find_sys(L, lt);                                       \
  const SysDesc* __restrict__ d = sys + L.sys[kk];                      \
  const int tile = lt - L.tile_begin[kk];                               \
  Scal* sc = L.scal + L.sys[kk];                                        \
  const Geom g = d->g;                                                  \
  const TileRange t_r = tile_range(tile, d->tnb, d->tbsz, d->tseg);     \
  const int t_lo = t_r.lo, t_hi = t_r.hi;                               \
  const int base = t_lo + threadIdx.x;                                  \
  (void)t_hi;                                                           \
  static_assert((TILE) > 0, "tile size");

// CG stage 1 of iteration it = L.it[kk]:
//   |r_it|^2 from the stage-2 partials of iteration it-1 (it > 0) and the stopping
//   test; p_new = r + beta p_old with beta = |r_it|^2 / |r_{it-1}|^2 (p_new = r at
//   it = 0), u = M^dagger p_new, partial of |u|^2 + mu^2 |p_new|^2 = <p, A p>.
// The loads of r and p_old are issued before the partial sums are read.
// The solution advances every second iteration (see k_cg2): a stage 1 that stops at
// an odd it adds the pending alpha_{it-1} p_{it-1} (p_old here) to x.  It marks the
// stop with active = 2 rather than 0 so that every workgroup of this launch still
// takes the stopping path; the next stage 2 sets 0.
template <typename C>
struct RP {
  C r, p;
};

template <typename R, typename LL, int SPT>
__global__ __launch_bounds__(kBlock) void k_cg1(const SysDesc* __restrict__ sys, LL L, int sR, int sP, int sU) {
  using C = typename V2<R>::T;
  constexpr int TILE = kBlock * SPT;
  HUB_PROLOGUE_T(TILE)
  if (!load_active(sc)) return;
  const int it = L.it[kk];
  const R mu2 = (R)d->mu2;
  const Vec<C> r(d->vec[sR]), po(d->vec[sP + (it & 1)]), pn(d->vec[sP + 1 - (it & 1)]), u(d->vec[sU]);
  const auto phi = phase_of<R>(d);
  R beta = 0;
  bool stopped = false;  // same value in every thread of every workgroup of the system
  // |r_it|^2, the stopping test and beta, once the stencil loads are in flight
  auto mid = [&]() -> bool {
    if (it == 0) return true;
    const double rr = sum_partials(d->part2, d->ntiles, 1);
    const double rr_prev = sc->rrv[(it - 1) & 1];
    const bool first = (tile == 0 && threadIdx.x == 0);
    if (!(rr > sc->stop2) || it >= sc->maxit) {
      if (first) {
        sc->rrv[it & 1] = rr;
        sc->iters = it;
        store_active(sc, 2);
      }
      stopped = true;
      return false;
    }
    if (first) sc->rrv[it & 1] = rr;
    beta = (R)(rr / rr_prev);
    return true;
  };
  R acc = 0;
  bool done = false;
  if constexpr (sizeof(R) == 4) {
    if ((g.L2 & 1) == 0) {
      auto pre2 = [](int) { return NoPre{}; };
      auto post2 = [&](int n, C64x2 uu, C64x2 p, NoPre) {
        pn.set_pair(n, p);
        u.set_pair(n, uu);
        acc += norm2<R>(uu.a) + norm2<R>(uu.b) + mu2 * (norm2<R>(p.a) + norm2<R>(p.b));
      };
      if (it == 0) {
        auto ld2 = [=](int k) { return r.pair(k); };
        auto ld1 = [=](int k) { return r[k]; };
        stencil_pairs<true, SPT>(g, phi, t_lo, t_hi, ld2, ld1, Same{}, Same{}, pre2, NoMid{}, post2);
      } else {
        auto ld2 = [=](int k) { return RP<C64x2>{r.pair(k), po.pair(k)}; };
        auto ld1 = [=](int k) { return RP<C>{r[k], po[k]}; };
        auto cook2 = [&](RP<C64x2> v) {
          C64x2 o;
          o.a.x = v.r.a.x + beta * v.p.a.x;
          o.a.y = v.r.a.y + beta * v.p.a.y;
          o.b.x = v.r.b.x + beta * v.p.b.x;
          o.b.y = v.r.b.y + beta * v.p.b.y;
          return o;
        };
        auto cook1 = [&](RP<C> v) {
          C o;
          o.x = v.r.x + beta * v.p.x;
          o.y = v.r.y + beta * v.p.y;
          return o;
        };
        stencil_pairs<true, SPT>(g, phi, t_lo, t_hi, ld2, ld1, cook2, cook1, pre2, mid, post2);
      }
      done = true;
    }
  }
  if (!done) {
    auto pre = [](int) { return NoPre{}; };
    auto post = [&](int n, C uu, C p, NoPre) {
      pn.set(n, p);
      u.set(n, uu);
      acc += norm2<R>(uu) + mu2 * norm2<R>(p);
    };
    if (it == 0) {
      auto ld = [=](int k) { return r[k]; };
      stencil_sites<R, true, Spt<R>::v, SPT>(g, phi, base, t_hi, ld, Same{}, pre, NoMid{}, post);
    } else {
      auto ld = [=](int k) { return RP<C>{r[k], po[k]}; };
      auto cook = [&](RP<C> v) {
        C o;
        o.x = v.r.x + beta * v.p.x;
        o.y = v.r.y + beta * v.p.y;
        return o;
      };
      stencil_sites<R, true, Spt<R>::v, SPT>(g, phi, base, t_hi, ld, cook, pre, mid, post);
    }
  }
  // a system that met its stopping test in `mid` writes no partial (none is read)
  if (stopped) {
    if (it & 1) {
      const R a = (R)sc->alpha[(it - 1) & 1];
      const Vec<C> x(d->vec[L.pi[kk]]);
      for (int k = base; k < t_hi; k += kBlock) {
        const C pv = po[k];
        C xv = x[k];
        xv.x = fma(a, pv.x, xv.x);
        xv.y = fma(a, pv.y, xv.y);
        x.set(k, xv);
      }
    }
    return;
  }
  const double tot = (double)block_sum(acc);
  if (threadIdx.x == 0) Real<double>(d->part1).set(tile, tot);
}

// CG stage 2 of iteration it: alpha = |r_it|^2 / <p, A p> (stage-1 partials),
// q = M u + mu^2 p, r -= alpha q, partial of |r_{it+1}|^2, and the solution every
// second iteration: x += alpha_{it-1} p_{it-1} + alpha_it p_it at odd it (p_{it-1}
// is still in the other slot of the pair), which saves a read and a write of x per
// two iterations for one read of p_{it-1}.  The solution slot of system k is L.pi[k].
// Loads are issued before alpha is read.  A system whose stage 1 stopped (active 2)
// does nothing here; workgroup 0 marks it stopped for good.
template <typename C, bool UPD>
struct Own {
  C p, r, x, q;  // x, q (p_{it-1}) loaded only when UPD
};
template <typename R, typename LL, int SPT>
__global__ __launch_bounds__(kBlock) void k_cg2(const SysDesc* __restrict__ sys, LL L, int sR, int sP, int sU) {
  using C = typename V2<R>::T;
  constexpr int TILE = kBlock * SPT;
  HUB_PROLOGUE_T(TILE)
  const int act = load_active(sc);
  if (act != 1) {
    if (act == 2 && tile == 0 && threadIdx.x == 0) store_active(sc, 0);
    return;
  }
  const int it = L.it[kk];
  R alpha = 0, alpha_prev = 0;
  auto mid = [&]() -> bool {
    const double pq = sum_partials(d->part1, d->ntiles, 1);
    const double a = sc->rrv[it & 1] / pq;
    if (tile == 0 && threadIdx.x == 0) sc->alpha[it & 1] = a;
    alpha = (R)a;
    if (it & 1) alpha_prev = (R)sc->alpha[(it - 1) & 1];
    return true;
  };
  const R mu2 = (R)d->mu2;
  const Vec<C> p(d->vec[sP + 1 - (it & 1)]), pp(d->vec[sP + (it & 1)]), u(d->vec[sU]), x(d->vec[L.pi[kk]]),
      r(d->vec[sR]);
  const auto phi = phase_of<R>(d);
  R acc = 0;
  auto run = [&](auto upd) {
    constexpr bool U = decltype(upd)::value;
    if constexpr (sizeof(R) == 4) {
      if ((g.L2 & 1) == 0) {
        auto ld2 = [=](int k) { return u.pair(k); };
        auto ld1 = [=](int k) { return u[k]; };
        auto pre2 = [=](int n) {
          Own<C64x2, U> o;
          o.p = p.pair(n);
          o.r = r.pair(n);
          if constexpr (U) {
            o.x = x.pair(n);
            o.q = pp.pair(n);
          }
          return o;
        };
        auto post2 = [&](int n, C64x2 q, C64x2, Own<C64x2, U> o) {
          C64x2 rv;
          rv.a.x = o.r.a.x - alpha * fma(mu2, o.p.a.x, q.a.x);
          rv.a.y = o.r.a.y - alpha * fma(mu2, o.p.a.y, q.a.y);
          rv.b.x = o.r.b.x - alpha * fma(mu2, o.p.b.x, q.b.x);
          rv.b.y = o.r.b.y - alpha * fma(mu2, o.p.b.y, q.b.y);
          r.set_pair(n, rv);
          if constexpr (U) {
            C64x2 xv;
            xv.a.x = fma(alpha, o.p.a.x, fma(alpha_prev, o.q.a.x, o.x.a.x));
            xv.a.y = fma(alpha, o.p.a.y, fma(alpha_prev, o.q.a.y, o.x.a.y));
            xv.b.x = fma(alpha, o.p.b.x, fma(alpha_prev, o.q.b.x, o.x.b.x));
            xv.b.y = fma(alpha, o.p.b.y, fma(alpha_prev, o.q.b.y, o.x.b.y));
            x.set_pair(n, xv);
          }
          acc += norm2<R>(rv.a) + norm2<R>(rv.b);
        };
        stencil_pairs<false, SPT>(g, phi, t_lo, t_hi, ld2, ld1, Same{}, Same{}, pre2, mid, post2);
        return;
      }
    }
    auto ld = [=](int k) { return u[k]; };
    auto pre = [=](int n) {
      Own<C, U> o;
      o.p = p[n];
      o.r = r[n];
      if constexpr (U) {
        o.x = x[n];
        o.q = pp[n];
      }
      return o;
    };
    auto post = [&](int n, C q, C, Own<C, U> o) {
      C rv;
      rv.x = o.r.x - alpha * fma(mu2, o.p.x, q.x);
      rv.y = o.r.y - alpha * fma(mu2, o.p.y, q.y);
      r.set(n, rv);
      if constexpr (U) {
        C xv;
        xv.x = fma(alpha, o.p.x, fma(alpha_prev, o.q.x, o.x.x));
        xv.y = fma(alpha, o.p.y, fma(alpha_prev, o.q.y, o.x.y));
        x.set(n, xv);
      }
      acc += norm2<R>(rv);
    };
    stencil_sites<R, false, Spt<R>::v, SPT>(g, phi, base, t_hi, ld, Same{}, pre, mid, post);
  };
  if (it & 1)
    run(std::true_type{});
  else
    run(std::false_type{});
  const double tot = (double)block_sum(acc);
  if (threadIdx.x == 0) Real<double>(d->part2).set(tile, tot);
}

// ---------------------------------------------------------------------------
// Single-workgroup complex64 CG for small systems, resident on one compute unit.
// One workgroup of kWgBlock threads owns a system of at most kWgMaxSites sites and
// runs up to K iterations of the same recurrence as k_cg1<float> / k_cg2<float> in one
// launch.  Each thread keeps r and the solution of its sites (threadIdx.x + m *
// kWgBlock, m < kWgPerThread) in registers, and the two vectors the stencil reads at
// neighbouring sites, p and u = M^dagger p, live in LDS (2 x 8 bytes x 10,200 sites
// fit in the 160 KB of a gfx950 CU); only the phase angles at the temporal neighbours
// are read from memory inside the loop.  Kernel boundaries become workgroup barriers
// and the reductions workgroup sums (wave64 butterflies, then the 16 wave results in
// a fixed order), so an iteration costs LDS traffic and two barriers instead of two
// launch floors and the vectors' round trips through L2.  An FP64 system of this size
// does not fit (p and u would take 2 x 16 bytes per site): FP64 CG keeps the tiled
// kernels.  The solution advances every iteration (x += alpha p).  Entry: r, x and
// p_old (slot S_P32 + (it & 1)) from memory; exit: the same slots written back,
// rrv[it & 1] = |r_it|^2, rrv[(it - 1) & 1] = |r_{it-1}|^2, and on a stop iters = it,
// active = 0.
// ---------------------------------------------------------------------------
// Sum over the workgroup in a fixed order; every thread gets the value.  `buf` holds one
// double per wave; callers alternate two buffers, so that the one barrier here also
// guarantees that the previous sum over the same buffer has been read by every thread
// (another barrier always separates two sums over one buffer).
template <typename T>
__device__ __forceinline__ double wg_sum(T v, double* buf) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) buf[threadIdx.x >> 6] = (double)v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kWgBlock / 64; ++k) s += buf[k];
  return s;
}

// Coordinates of the sites n0 + m * step, m = 0, 1, ...: one division pair for m = 0, then
// a step of `step` sites per m (dj columns, then di rows and dq planes with one carry each:
// di + 1 <= L1 and dj < L2 keep every carry to one subtraction).
struct WgWalk {
  int i, j;
  uint32_t q2;
  int dj, di, dq;
  __device__ __forceinline__ void next(const Geom& g) {
    j += dj;
    const int cj = j >= g.L2;
    j -= cj * g.L2;
    i += di + cj;
    const int ci = i >= g.L1;
    i -= ci * g.L1;
    q2 += (uint32_t)(dq + ci);
  }
};

__device__ __forceinline__ WgWalk wg_walk(const Geom& g, int n0, int step) {
  WgWalk w;
  const uint32_t q1 = fdiv((uint32_t)n0, g.dL2);
  w.j = n0 - (int)q1 * g.L2;
  w.q2 = fdiv(q1, g.dL1);
  w.i = (int)q1 - (int)w.q2 * g.L1;
  const int rows = step / g.L2;  // whole rows in a step
  w.dj = step - rows * g.L2;
  w.dq = rows / g.L1;
  w.di = rows - w.dq * g.L1;
  // the start is laundered so that the walk is redone in every pass rather than hoisted
  // out of the iteration loop, where its ten sites' coordinates would not fit in registers
  asm volatile("" : "+v"(w.i), "+v"(w.j), "+v"(w.q2));
  return w;
}

// (cos, sin) of row h of a pair of precomputed phases.
__device__ __forceinline__ void pick(const C64x2& e, int h, float& c, float& s) {
  c = h ? e.b.x : e.a.x;
  s = h ? e.b.y : e.a.y;
}

// Pair view of an LDS array of complex64 values: sites k, k + 1 (k even) in one 16-byte
// access.
__device__ __forceinline__ C64x2 lds_pair(const float2* a, int k) {
  const hub_f4v v = reinterpret_cast<const hub_f4v*>(a)[k >> 1];
  C64x2 r;
  r.a.x = v.x;
  r.a.y = v.y;
  r.b.x = v.z;
  r.b.y = v.w;
  return r;
}
__device__ __forceinline__ void lds_set_pair(float2* a, int k, C64x2 v) {
  hub_f4v w;
  w.x = v.a.x;
  w.y = v.a.y;
  w.z = v.b.x;
  w.w = v.b.y;
  reinterpret_cast<hub_f4v*>(a)[k >> 1] = w;
}

// The iterations of one system.  PAIR (even L2): each thread owns the site pairs
// (2u, 2u + 1), u = threadIdx.x + m * kWgBlock, and applies the stencil a pair at a time
// (index arithmetic once per pair, 16-byte LDS accesses); otherwise the single sites
// threadIdx.x + m * kWgBlock.  Site k of unit m sits in rv[m * S + k] etc., S sites per unit.
template <bool PAIR, bool CSL>
__device__ __forceinline__ void wg_cg(const SysDesc* __restrict__ d, Scal* sc, const WgList& L, int kk, int K,
                                      float2* __restrict__ lp, float2* __restrict__ lu, float2* __restrict__ lc,
                                      double (*red)[kWgBlock / 64]) {
  constexpr int S = PAIR ? 2 : 1;
  constexpr int U = kWgPerThread / S;  // units per thread
  const int u0 = S * (int)threadIdx.x, ustep = S * kWgBlock;
  const Geom g = d->g;
  const int N = g.n;
  const int it0 = L.it[kk];
  const float mu2 = (float)d->mu2;
  const double stop2 = sc->stop2;
  const int maxit = sc->maxit;
  const Vec<float2> r(d->vec[S_R32]), x(d->vec[L.pi[kk]]), cs(d->cs32);
  float2 rv[kWgPerThread], xv[kWgPerThread], ev[kWgPerThread];  // ev: (cos, sin) of the own site
  {
    const Vec<float2> po(d->vec[S_P32 + (it0 & 1)]);
#pragma unroll
    for (int m = 0; m < U; ++m) {
      const int n = u0 + m * ustep;
      if (n < N) {
        if constexpr (PAIR) {
          const C64x2 a = r.pair(n), b = x.pair(n), e = cs.pair(n);
          rv[2 * m] = a.a;
          rv[2 * m + 1] = a.b;
          xv[2 * m] = b.a;
          xv[2 * m + 1] = b.b;
          ev[2 * m] = e.a;
          ev[2 * m + 1] = e.b;
          if (it0 > 0) lds_set_pair(lp, n, po.pair(n));
        } else {
          rv[m] = r[n];
          xv[m] = x[n];
          ev[m] = cs[n];
          if (it0 > 0) lp[n] = po[n];
        }
      }
    }
  }
  if constexpr (CSL)
    for (int n = threadIdx.x; n < N; n += kWgBlock) lc[n] = cs[n];
  double rr = sc->rrv[it0 & 1];
  double rr_prev = it0 > 0 ? sc->rrv[(it0 - 1) & 1] : 1.0;
  int it = it0;
  bool stopped = false;
  __syncthreads();
  for (int step = 0; step < K; ++step, ++it) {
    // the stopping test of iteration it (at it = 0 the CG setup decided)
    if (it > 0 && (!(rr > stop2) || it >= maxit)) {
      stopped = true;
      break;
    }
    const float beta = it == 0 ? 0.0f : (float)(rr / rr_prev);
    float acc = 0.0f;
    // p = r + beta p_old on this thread's sites
#pragma unroll
    for (int m = 0; m < U; ++m) {
      const int n = u0 + m * ustep;
      if (n < N) {
        if constexpr (PAIR) {
          C64x2 pv;
          pv.a = rv[2 * m];
          pv.b = rv[2 * m + 1];
          if (it > 0) {
            const C64x2 q = lds_pair(lp, n);
            pv.a.x = fmaf(beta, q.a.x, pv.a.x);
            pv.a.y = fmaf(beta, q.a.y, pv.a.y);
            pv.b.x = fmaf(beta, q.b.x, pv.b.x);
            pv.b.y = fmaf(beta, q.b.y, pv.b.y);
          }
          lds_set_pair(lp, n, pv);
          acc += mu2 * (norm2<float>(pv.a) + norm2<float>(pv.b));
        } else {
          float2 pv = rv[m];
          if (it > 0) {
            const float2 q = lp[n];
            pv.x = fmaf(beta, q.x, pv.x);
            pv.y = fmaf(beta, q.y, pv.y);
          }
          lp[n] = pv;
          acc += mu2 * norm2<float>(pv);
        }
      }
    }
    __syncthreads();
    // u = M^dagger p (the phase of the temporal neighbour, from the table); <p, A p> =
    // |u|^2 + mu2 |p|^2
    {
      WgWalk wk = wg_walk(g, u0, ustep);
#pragma unroll
      for (int m = 0; m < U; ++m) {
        const int n = u0 + m * ustep;
        if (n < N) {
          if constexpr (PAIR) {
            const PairIdx sm = pair_index_at<true>(g, n, wk.i, wk.j, wk.q2);
            const C64x2 e = CSL ? lds_pair(lc, sm.tn) : cs.pair(sm.tn);
            const C64x2 y = pair_stencil<true>(g, sm, [&](int h, float& c, float& s) { pick(e, h, c, s); },
                                               lds_pair(lp, n), lds_pair(lp, sm.tn), lds_pair(lp, sm.h0),
                                               lds_pair(lp, sm.h1), lp[sm.hx]);
            lds_set_pair(lu, n, y);
            acc += norm2<float>(y.a) + norm2<float>(y.b);
          } else {
            const SiteIdx st = site_index_at<true>(g, n, wk.i, wk.j, wk.q2);
            const float2 e = CSL ? lc[st.pn] : cs[st.pn];
            const float2 xs = lp[st.n], xt = lp[st.tn], x0 = lp[st.h0], x1 = lp[st.h1], x2 = lp[st.h2];
            const float2 y = stencil_combine<float, true>(g, st, e.x, e.y, xs, xt, x0, x1, x2);
            lu[n] = y;
            acc += norm2<float>(y);
          }
        }
        wk.next(g);
      }
    }
    // FP32 sums within a wave (as the tiled kernels' workgroup sums), FP64 across waves
    const double pap = wg_sum(acc, red[0]);  // its barrier also publishes u
    const float alpha = (float)(rr / pap);
    // q = M u + mu2 p; r -= alpha q; x += alpha p; |r|^2
    float acc2 = 0.0f;
    {
      WgWalk wk = wg_walk(g, u0, ustep);
#pragma unroll
      for (int m = 0; m < U; ++m) {
        const int n = u0 + m * ustep;
        if (n < N) {
          float2 q[S], pv[S];
          if constexpr (PAIR) {
            const PairIdx sm = pair_index_at<false>(g, n, wk.i, wk.j, wk.q2);
            C64x2 e;
            e.a = ev[2 * m];
            e.b = ev[2 * m + 1];
            const C64x2 y = pair_stencil<false>(g, sm, [&](int h, float& c, float& s) { pick(e, h, c, s); },
                                                lds_pair(lu, n), lds_pair(lu, sm.tn), lds_pair(lu, sm.h0),
                                                lds_pair(lu, sm.h1), lu[sm.hx]);
            const C64x2 pp = lds_pair(lp, n);
            q[0] = y.a;
            q[S - 1] = y.b;
            pv[0] = pp.a;
            pv[S - 1] = pp.b;
          } else {
            const SiteIdx st = site_index_at<false>(g, n, wk.i, wk.j, wk.q2);
            const float2 xs = lu[st.n], xt = lu[st.tn], x0 = lu[st.h0], x1 = lu[st.h1], x2 = lu[st.h2];
            q[0] = stencil_combine<float, false>(g, st, ev[m].x, ev[m].y, xs, xt, x0, x1, x2);
            pv[0] = lp[n];
          }
#pragma unroll
          for (int h = 0; h < S; ++h) {
            float2& rk = rv[m * S + h];
            float2& xk = xv[m * S + h];
            rk.x -= alpha * fmaf(mu2, pv[h].x, q[h].x);
            rk.y -= alpha * fmaf(mu2, pv[h].y, q[h].y);
            xk.x = fmaf(alpha, pv[h].x, xk.x);
            xk.y = fmaf(alpha, pv[h].y, xk.y);
            acc2 += norm2<float>(rk);
          }
        }
        wk.next(g);
      }
    }
    rr_prev = rr;
    rr = wg_sum(acc2, red[1]);
  }
  // write the state back: r, x, and p_{it-1} to the slot iteration `it` reads it from
  {
    const Vec<float2> pw(d->vec[S_P32 + (it & 1)]);
#pragma unroll
    for (int m = 0; m < U; ++m) {
      const int n = u0 + m * ustep;
      if (n < N) {
        if constexpr (PAIR) {
          C64x2 a, b;
          a.a = rv[2 * m];
          a.b = rv[2 * m + 1];
          b.a = xv[2 * m];
          b.b = xv[2 * m + 1];
          r.set_pair(n, a);
          x.set_pair(n, b);
          if (it > 0) pw.set_pair(n, lds_pair(lp, n));
        } else {
          r.set(n, rv[m]);
          x.set(n, xv[m]);
          if (it > 0) pw.set(n, lp[n]);
        }
      }
    }
  }
  if (threadIdx.x == 0) {
    sc->rrv[it & 1] = rr;
    if (it > 0) sc->rrv[(it - 1) & 1] = rr_prev;
    if (stopped) {
      sc->iters = it;
      store_active(sc, 0);
    }
  }
}

__global__ __launch_bounds__(kWgBlock) void k_cg_wg32(const SysDesc* __restrict__ sys, WgList L, int K) {
  extern __shared__ __attribute__((aligned(16))) float2 wlds[];  // p [nmax], u [nmax] (nmax even), cs [nmax]
  const int kk = blockIdx.x;
  const SysDesc* __restrict__ d = sys + L.sys[kk];
  Scal* sc = L.scal + L.sys[kk];
  if (!load_active(sc)) return;
  float2* __restrict__ lp = wlds;
  float2* __restrict__ lu = wlds + L.nmax;
  float2* __restrict__ lc = wlds + 2 * L.nmax;
  __shared__ double red[2][kWgBlock / 64];  // the two alternating buffers of wg_sum
  if ((d->g.L2 & 1) == 0) {
    if (L.cs_lds)
      wg_cg<true, true>(d, sc, L, kk, K, lp, lu, lc, red);
    else
      wg_cg<true, false>(d, sc, L, kk, K, lp, lu, lc, red);
  } else {
    if (L.cs_lds)
      wg_cg<false, true>(d, sc, L, kk, K, lp, lu, lc, red);
    else
      wg_cg<false, false>(d, sc, L, kk, K, lp, lu, lc, red);
  }
}

// ---------------------------------------------------------------------------
// Multi-shift CG (FP64).  Base CG on A_0 as k_cg1 / k_cg2; every shifted system s
// follows with x_s += alpha^s_k p^s_k, p^s_{k+1} = zeta^s_{k+1} r_{k+1} + beta^s_k p^s_k,
//   zeta^s_{k+1} = zeta_k zeta_{k-1} alpha_{k-1} /
//                  (alpha_k beta_{k-1} (zeta_{k-1} - zeta_k) + zeta_{k-1} alpha_{k-1} (1 + sigma_s alpha_k)),
//   alpha^s_k = alpha_k zeta_{k+1} / zeta_k,  beta^s_k = beta_k (zeta_{k+1} / zeta_k)^2,
// until its residual |zeta^s| |r| meets the tolerance.  Every workgroup evaluates the
// scalar recurrences in the same order (one thread per shift), so they agree.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_ms_start(const MsDesc* __restrict__ d) {
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const TileRange tr = tile_range(tile, d->tnb, d->tbsz, d->tseg);
  const int base = tr.lo + threadIdx.x;
  double acc = 0.0;
  const double2 z = {0.0, 0.0};
  for (int m = 0; m < kSitesPerThread; ++m) {
    const int n = base + m * kBlock;
    if (n >= tr.hi) break;
    const double2 v = d->b[n];
    d->r[n] = v;
    d->x[n] = z;
    for (int s = 0; s < d->ns; ++s) {
      d->xs[s][n] = z;
      d->ps[s][n] = v;
    }
    acc += v.x * v.x + v.y * v.y;
  }
  const double tot = block_sum(acc);
  if (threadIdx.x == 0) d->part2[tile] = tot;
}

__global__ __launch_bounds__(kBlock) void k_ms_setup(const MsDesc* __restrict__ d) {
  const double rr = sum_partials(d->part2, d->ntiles, 1);
  if (threadIdx.x == 0) {
    MsScal* sc = d->sc;
    sc->rrv[0] = rr;
    sc->rrv[1] = rr;
    sc->alpha[0] = 1.0;
    sc->alpha[1] = 1.0;
    sc->beta[0] = 0.0;
    sc->beta[1] = 0.0;
    sc->stop2 = d->tol2 * rr;
    for (int s = 0; s < kMsMax; ++s) {
      sc->zeta[s][0] = sc->zeta[s][1] = sc->zeta[s][2] = 1.0;
      sc->frozen[s][0] = sc->frozen[s][1] = 0;
    }
    sc->iters = 0;
    sc->maxit = d->maxit;
    sc->stop = 0;
    __hip_atomic_store(&sc->active, rr > 0.0 ? 1 : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__device__ __forceinline__ int ms_load_active(MsScal* sc) {
  return __hip_atomic_load(&sc->active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Stage 1 of iteration it: |r_it|^2, beta_{it-1}, the shifted scalars of step it-1 and
// the stopping test; p_it = r_it + beta p_{it-1}, u = M^dagger p_it, partial <p, A_0 p>;
// then the shifted vector updates of step it-1 (also in the iteration that stops).
__global__ __launch_bounds__(kBlock) void k_ms1(const MsDesc* __restrict__ d, int it) {
  MsScal* sc = d->sc;
  if (!ms_load_active(sc)) return;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const Geom g = d->g;
  const TileRange tr = tile_range(tile, d->tnb, d->tbsz, d->tseg);
  const int base = tr.lo + threadIdx.x;
  const double mu2 = d->mu2;
  const int ns = d->ns;
  const Vec<double2> r(d->r), po(d->p[it & 1]), pn(d->p[1 - (it & 1)]), u(d->u);
  const PhasePhi<double> phi(d->ph64);
  __shared__ double s_as[kMsMax], s_bs[kMsMax], s_zn[kMsMax];
  __shared__ int s_live[kMsMax];
  double beta = 0.0;
  bool stopped = false;
  auto mid = [&]() -> bool {
    const double rr = sum_partials(d->part2, d->ntiles, 1);
    const double rr_prev = sc->rrv[(it - 1) & 1];
    beta = rr / rr_prev;
    const int k = it - 1;
    const double a_k = sc->alpha[k & 1], a_km = sc->alpha[(k + 1) & 1], b_km = sc->beta[(k + 1) & 1];
    if ((int)threadIdx.x < ns) {
      const int s = threadIdx.x;
      const bool live = sc->frozen[s][k & 1] == 0;
      const double zk = sc->zeta[s][k % 3], zkm = sc->zeta[s][(k + 2) % 3];
      double zn = zk, as = 0.0, bs = 1.0;
      if (live) {
        zn = zk * zkm * a_km / (a_k * b_km * (zkm - zk) + zkm * a_km * (1.0 + d->sigma[s] * a_k));
        as = a_k * zn / zk;
        bs = beta * (zn / zk) * (zn / zk);
      }
      s_as[s] = as;
      s_bs[s] = bs;
      s_zn[s] = zn;
      s_live[s] = live ? 1 : 0;
      if (tile == 0) {
        sc->zeta[s][(k + 1) % 3] = zn;
        sc->frozen[s][(k + 1) & 1] = (!live || zn * zn * rr <= sc->stop2) ? 1 : 0;
      }
    }
    __syncthreads();
    const bool first = (tile == 0 && threadIdx.x == 0);
    if (first) {
      sc->rrv[it & 1] = rr;
      sc->beta[k & 1] = beta;
      d->hist[2 * k + 1] = beta;
    }
    if (!(rr > sc->stop2) || it >= sc->maxit) {
      // every workgroup of this launch still runs (active stays set until the next
      // stage 2), so all of them apply the last shifted updates below
      if (first) {
        sc->iters = it;
        sc->stop = 1;
      }
      stopped = true;
      return false;
    }
    return true;
  };
  double acc = 0.0;
  auto pre = [](int) { return NoPre{}; };
  auto post = [&](int n, double2 uu, double2 p, NoPre) {
    pn.set(n, p);
    u.set(n, uu);
    acc += norm2<double>(uu) + mu2 * norm2<double>(p);
  };
  if (it == 0) {
    auto ld = [=](int k) { return r[k]; };
    stencil_sites<double, true, HUB_SPT64>(g, phi, base, tr.hi, ld, Same{}, pre, NoMid{}, post);
  } else {
    auto ld = [=](int k) { return RP<double2>{r[k], po[k]}; };
    auto cook = [&](RP<double2> v) {
      double2 o;
      o.x = v.r.x + beta * v.p.x;
      o.y = v.r.y + beta * v.p.y;
      return o;
    };
    stencil_sites<double, true, HUB_SPT64>(g, phi, base, tr.hi, ld, cook, pre, mid, post);
    // shifted systems, step it-1 -> it
    for (int m = 0; m < kSitesPerThread; ++m) {
      const int n = base + m * kBlock;
      if (n >= tr.hi) break;
      const double2 rv = r[n];
      for (int s = 0; s < ns; ++s) {
        if (!s_live[s]) continue;
        const Vec<double2> xs(d->xs[s]), ps(d->ps[s]);
        const double2 pv = ps[n];
        double2 xv = xs[n];
        xv.x += s_as[s] * pv.x;
        xv.y += s_as[s] * pv.y;
        double2 q;
        q.x = s_zn[s] * rv.x + s_bs[s] * pv.x;
        q.y = s_zn[s] * rv.y + s_bs[s] * pv.y;
        xs.set(n, xv);
        ps.set(n, q);
      }
    }
  }
  if (stopped) return;
  const double tot = block_sum(acc);
  if (threadIdx.x == 0) Real<double>(d->part1).set(tile, tot);
}

// Stage 2 of iteration it: alpha_it = |r_it|^2 / <p, A_0 p>, q = M u + mu2 p,
// x += alpha p, r -= alpha q, partial |r_{it+1}|^2.
__global__ __launch_bounds__(kBlock) void k_ms2(const MsDesc* __restrict__ d, int it) {
  MsScal* sc = d->sc;
  if (!ms_load_active(sc)) return;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  if (sc->stop) {
    if (tile == 0 && threadIdx.x == 0)
      __hip_atomic_store(&sc->active, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  const Geom g = d->g;
  const TileRange tr = tile_range(tile, d->tnb, d->tbsz, d->tseg);
  const int base = tr.lo + threadIdx.x;
  const double mu2 = d->mu2;
  double alpha = 0.0;
  auto mid = [&]() -> bool {
    const double pq = sum_partials(d->part1, d->ntiles, 1);
    alpha = sc->rrv[it & 1] / pq;
    if (tile == 0 && threadIdx.x == 0) {
      sc->alpha[it & 1] = alpha;
      d->hist[2 * it] = alpha;
    }
    return true;
  };
  const Vec<double2> p(d->p[1 - (it & 1)]), u(d->u), x(d->x), r(d->r);
  const PhasePhi<double> phi(d->ph64);
  struct Own {
    double2 p, x, r;
  };
  double acc = 0.0;
  auto ld = [=](int k) { return u[k]; };
  auto pre = [=](int n) { return Own{p[n], x[n], r[n]}; };
  auto post = [&](int n, double2 q, double2, Own o) {
    q.x += mu2 * o.p.x;
    q.y += mu2 * o.p.y;
    double2 xv = o.x, rv = o.r;
    xv.x += alpha * o.p.x;
    xv.y += alpha * o.p.y;
    rv.x -= alpha * q.x;
    rv.y -= alpha * q.y;
    x.set(n, xv);
    r.set(n, rv);
    acc += norm2<double>(rv);
  };
  stencil_sites<double, false, HUB_SPT64>(g, phi, base, tr.hi, ld, Same{}, pre, mid, post);
  const double tot = block_sum(acc);
  if (threadIdx.x == 0) Real<double>(d->part2).set(tile, tot);
}

template <typename Tin> __device__ __forceinline__ double2 to_c128(Tin v);
template <> __device__ __forceinline__ double2 to_c128<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ double2 to_c128<float2>(float2 v) {
  double2 o;
  o.x = v.x;
  o.y = v.y;
  return o;
}




__device__ __forceinline__ void store_partials(const SysDesc* d, int tile, const double* vals, int nv) {
  if (threadIdx.x == 0) {
    const Real<double> p(d->part + (size_t)tile * kMaxRed);
    for (int q = 0; q < nv; ++q) p.set(q, vals[q]);
  }
}

// ---------------------------------------------------------------------------
// The normal operator A = M M^dagger + mu2 in one pass.  From eq. (ferm_op), with
// c_A(t) = s(t) (e^{i phi_A(t)} - m) and c_B(t) = s'(t) (e^{-i phi_B(t)} - m) (s = -1
// on the A hop out of t = 0, s' = -1 on the B hop out of t = N_t - 1), the same-slice
// A-B terms of M M^dagger cancel and each row has 12 entries:
//   A(t): (1 + |c_A(t)|^2 + 3 kappa^2 + mu2) x - c_A(t) x_A(t-1) - conj(c_A(t+1)) x_A(t+1)
//         + kappa^2 sum_6 x_A(t) - kappa sum_b (c_A(t) - conj(c_B(t-1)[b])) x_B(t-1)[b]
//   B(t): (1 + |c_B(t)|^2 + 3 kappa^2 + mu2) x - c_B(t) x_B(t+1) - conj(c_B(t-1)) x_B(t-1)
//         + kappa^2 sum_6 x_B(t) - kappa sum_a (conj(c_A(t+1)[a]) - c_B(t)) x_A(t+1)[a]
// where sum_6 runs over the second neighbours (i, j) + {(1,0), (0,1), (-1,0), (-1,1),
// (0,-1), (1,-1)} (the A-B-A and B-A-B paths; wrapped offsets that coincide add,
// exactly as the paths do) and b / a over the three bonds of the site (at slice
// t-1 for A rows, t+1 for B rows).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  double2 r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) b
  double2 r;
  r.x = a.x * b.x + a.y * b.y;
  r.y = a.x * b.y - a.y * b.x;
  return r;
}

template <typename Load>
__device__ __forceinline__ double2 normal12(const Geom& g, const PhasePhi<double>& ph, int n, double mu2, Load ld) {
  const uint32_t q1 = fdiv((uint32_t)n, g.dL2);
  const int j = n - (int)q1 * g.L2;
  const uint32_t q2 = fdiv(q1, g.dL1);
  const int i = (int)q1 - (int)q2 * g.L1;
  const bool isA = (q2 & 1u) == 0;
  const int t = (int)(q2 >> 1);
  const int P = g.P, L1 = g.L1, L2 = g.L2;
  const int tp = (t + 1 == g.Nt) ? 0 : t + 1, tm = (t == 0) ? g.Nt - 1 : t - 1;
  const int ip = (i + 1 == L1) ? 0 : i + 1, im = (i == 0) ? L1 - 1 : i - 1;
  const int jp = (j + 1 == L2) ? 0 : j + 1, jm = (j == 0) ? L2 - 1 : j - 1;
  const int r0 = i * L2, rp = ip * L2, rm = im * L2;
  const int own = n;
  const int pA = 2 * t * P, pB = pA + P;                // planes of slice t
  const int here = isA ? pA : pB;
  // same sublattice at t-1, t+1
  const int nm = (isA ? 2 * tm * P : 2 * tm * P + P) + r0 + j;
  const int np = (isA ? 2 * tp * P : 2 * tp * P + P) + r0 + j;
  // opposite sublattice: A rows take B at t-1 (bonds (i,j), (i-1,j), (i,j-1));
  // B rows take A at t+1 (bonds (i,j), (i+1,j), (i,j+1))
  const int ob = isA ? 2 * tm * P + P : 2 * tp * P;
  const int b0 = ob + r0 + j;
  const int b1 = isA ? ob + rm + j : ob + rp + j;
  const int b2 = isA ? ob + r0 + jm : ob + r0 + jp;
  const double2 xs = ld(own), xm = ld(nm), xp = ld(np);
  const double2 s0 = ld(here + rp + j), s1 = ld(here + r0 + jp), s2 = ld(here + rm + j);
  const double2 s3 = ld(here + rm + jp), s4 = ld(here + r0 + jm), s5 = ld(here + rp + jm);
  const double2 y0 = ld(b0), y1 = ld(b1), y2 = ld(b2);
  const double2 e_own = ph.p[own];
  const double2 e_t = ph.p[isA ? np : nm];  // A: c_A(t+1); B: c_B(t-1)
  const double2 e0 = ph.p[b0], e1 = ph.p[b1], e2 = ph.p[b2];
  const double m = g.ms, kap = g.kappa;
  // signs of the hops: A hop out of slice u carries -1 iff u = 0; B hop iff u = N_t - 1
  const double sA_t = (t == 0) ? -1.0 : 1.0, sA_tp = (t == g.Nt - 1) ? -1.0 : 1.0;
  const double sB_t = (t == g.Nt - 1) ? -1.0 : 1.0, sB_tm = (t == 0) ? -1.0 : 1.0;
  auto cA = [&](double2 e, double sg) { double2 c; c.x = sg * (e.x - m); c.y = sg * e.y; return c; };
  auto cB = [&](double2 e, double sg) { double2 c; c.x = sg * (e.x - m); c.y = -sg * e.y; return c; };
  double2 c_own, c_t, k0, k1, k2;
  if (isA) {
    c_own = cA(e_own, sA_t);                 // c_A(t)
    c_t = cA(e_t, sA_tp);                    // c_A(t+1)
    const double2 d0 = cB(e0, sB_tm), d1 = cB(e1, sB_tm), d2 = cB(e2, sB_tm);  // c_B(t-1)[b]
    k0.x = c_own.x - d0.x; k0.y = c_own.y + d0.y;   // c_A(t) - conj(c_B)
    k1.x = c_own.x - d1.x; k1.y = c_own.y + d1.y;
    k2.x = c_own.x - d2.x; k2.y = c_own.y + d2.y;
  } else {
    c_own = cB(e_own, sB_t);                 // c_B(t)
    c_t = cB(e_t, sB_tm);                    // c_B(t-1)
    const double2 d0 = cA(e0, sA_tp), d1 = cA(e1, sA_tp), d2 = cA(e2, sA_tp);  // c_A(t+1)[a]
    k0.x = d0.x - c_own.x; k0.y = -d0.y - c_own.y;  // conj(c_A) - c_B(t)
    k1.x = d1.x - c_own.x; k1.y = -d1.y - c_own.y;
    k2.x = d2.x - c_own.x; k2.y = -d2.y - c_own.y;
  }
  const double diag = 1.0 + c_own.x * c_own.x + c_own.y * c_own.y + 3.0 * kap * kap + mu2;
  // temporal: A: - c_A(t) x(t-1) - conj(c_A(t+1)) x(t+1);  B: - c_B(t) x(t+1) - conj(c_B(t-1)) x(t-1)
  const double2 ta = cmul(c_own, isA ? xm : xp);
  const double2 tb = cmulc(c_t, isA ? xp : xm);
  const double2 bo0 = cmul(k0, y0), bo1 = cmul(k1, y1), bo2 = cmul(k2, y2);
  const double k2s = kap * kap;
  double2 q;
  q.x = diag * xs.x - ta.x - tb.x + k2s * (s0.x + s1.x + s2.x + s3.x + s4.x + s5.x) - kap * (bo0.x + bo1.x + bo2.x);
  q.y = diag * xs.y - ta.y - tb.y + k2s * (s0.y + s1.y + s2.y + s3.y + s4.y + s5.y) - kap * (bo0.y + bo1.y + bo2.y);
  return q;
}

// out = [b -] (M M^dagger + mu2) in, FP64 arithmetic (in: FP64 or complex64 slot),
// partial |out|^2 (mode != RED_NONE).  One pass of the 12-point form.
template <typename Tin, int SPT>
__global__ __launch_bounds__(kBlock) void k_normal_slot(const SysDesc* __restrict__ sys, LaunchList L, int s_in,
                                                        int s_b, int s_out, int mode) {
  constexpr int TILE = kBlock * SPT;
  HUB_PROLOGUE_T(TILE)
  (void)sc;
  const Vec<Tin> in(d->vec[s_in]);
  const bool has_b = s_b >= 0;
  const Vec<double2> bv(has_b ? d->vec[s_b] : nullptr), out(d->vec[s_out]);
  const PhasePhi<double> ph = phase_of<double>(d);
  const double mu2 = d->mu2;
  auto ld = [=](int k) { return to_c128<Tin>(in[k]); };
  double acc = 0.0;
#pragma unroll 2
  for (int m = 0; m < SPT; ++m) {
    const int n = base + m * kBlock;
    if (n >= t_hi) break;
    double2 q = normal12(g, ph, n, mu2, ld);
    if (has_b) {
      const double2 bb = bv[n];
      q.x = bb.x - q.x;
      q.y = bb.y - q.y;
    }
    out.set(n, q);
    acc += norm2<double>(q);
  }
  if (mode == RED_NONE) return;
  const double tot = block_sum(acc);
  store_partials(d, tile, &tot, 1);
}



// x = 0, r = b; partial of |b|^2, made NaN where the phase of phi is not finite (so
// that a non-finite phi or b shows in the first reduction the host reads).
template <int SPT>
__global__ __launch_bounds__(kBlock) void k_cg_init_zero(const SysDesc* __restrict__ sys, LaunchList L) {
  constexpr int TILE = kBlock * SPT;
  HUB_PROLOGUE_T(TILE)
  (void)sc;
  const Vec<double2> b(d->vec[S_B]), x(d->vec[S_X]), r(d->vec[S_R]), ph(d->ph64);
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < SPT; ++m) {
    const int n = base + m * kBlock;
    if (n < t_hi) {
      const double2 v = b[n];
      const double2 e = ph[n];
      r.set(n, v);
      x.set(n, cz<double2>());
      acc += norm2<double>(v);
      if (!isfinite(e.x) || !isfinite(e.y)) acc = __builtin_nan("");
    }
  }
  const double tot = block_sum(acc);
  store_partials(d, tile, &tot, 1);
}

// partials of <v_i, w> = sum conj(v_i) w, i < cnt (re, im interleaved).
template <int SPT>
__global__ __launch_bounds__(kBlock) void k_multidot(const SysDesc* __restrict__ sys, LaunchList L, int s_w,
                                                     int s_v0, int cnt) {
  constexpr int TILE = kBlock * SPT;
  HUB_PROLOGUE_T(TILE)
  (void)sc;
  const Vec<double2> w(d->vec[s_w]);
  double2 wv[SPT];
#pragma unroll
  for (int m = 0; m < SPT; ++m) {
    const int n = base + m * kBlock;
    wv[m] = cz<double2>();
    if (n < t_hi) wv[m] = w[n];
  }
  __shared__ double tot[kMaxRed];
  for (int q = 0; q < cnt; ++q) {
    const Vec<double2> v(d->vec[s_v0 + q]);
    double ar = 0.0, ai = 0.0;
#pragma unroll
    for (int m = 0; m < SPT; ++m) {
      const int n = base + m * kBlock;
      if (n < t_hi) {
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
  store_partials(d, tile, tot, 2 * cnt);
}

// w -= sum_i h_i v_i, h_i = red[h_off + 2i] + i red[h_off + 2i + 1]; partial of |w|^2.
template <int SPT>
__global__ __launch_bounds__(kBlock) void k_cgs(const SysDesc* __restrict__ sys, LaunchList L, int s_w, int s_v0,
                                                int cnt, int h_off) {
  constexpr int TILE = kBlock * SPT;
  HUB_PROLOGUE_T(TILE)
  const Vec<double2> w(d->vec[s_w]);
  double2 wv[SPT];
#pragma unroll
  for (int m = 0; m < SPT; ++m) {
    const int n = base + m * kBlock;
    wv[m] = cz<double2>();
    if (n < t_hi) wv[m] = w[n];
  }
  for (int q = 0; q < cnt; ++q) {
    const double hr = sc->red[h_off + 2 * q], hi = sc->red[h_off + 2 * q + 1];
    const Vec<double2> v(d->vec[s_v0 + q]);
#pragma unroll
    for (int m = 0; m < SPT; ++m) {
      const int n = base + m * kBlock;
      if (n < t_hi) {
        const double2 vv = v[n];
        wv[m].x -= hr * vv.x - hi * vv.y;
        wv[m].y -= hr * vv.y + hi * vv.x;
      }
    }
  }
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < SPT; ++m) {
    const int n = base + m * kBlock;
    if (n < t_hi) {
      w.set(n, wv[m]);
      acc += norm2<double>(wv[m]);
    }
  }
  const double tot = block_sum(acc);
  store_partials(d, tile, &tot, 1);
}

// v = pa*src (FP64, stored to s_v if s_v >= 0).  With pi = maxit > 0 the
// single-precision CG starts on v: r32 = c64(v), z = 0, partial of |r32|^2 (FP32
// sums).  With pi = 0 there is no preconditioning: z = c64(v).  The z slot of
// system k is pj[k].
template <int SPT>
__global__ __launch_bounds__(kBlock) void k_prep_inner(const SysDesc* __restrict__ sys, LaunchList L, int s_src,
                                                       int s_v) {
  constexpr int TILE = kBlock * SPT;
  HUB_PROLOGUE_T(TILE)
  (void)sc;
  const double scale = L.pa[kk];
  const int maxit = L.pi[kk];
  const bool store_v = s_v >= 0;
  const Vec<double2> src(d->vec[s_src]), v(store_v ? d->vec[s_v] : nullptr);
  const Vec<float2> z(d->vec[L.pj[kk]]), r32(d->vec[S_R32]);
  float acc = 0.0f;
#pragma unroll
  for (int m = 0; m < SPT; ++m) {
    const int n = base + m * kBlock;
    if (n < t_hi) {
      double2 a = src[n];
      a.x *= scale;
      a.y *= scale;
      if (store_v) v.set(n, a);
      float2 a32;
      a32.x = (float)a.x;
      a32.y = (float)a.y;
      if (maxit > 0) {
        r32.set(n, a32);
        z.set(n, cz<float2>());
        acc += norm2<float>(a32);
      } else {
        z.set(n, a32);
      }
    }
  }
  if (maxit <= 0) return;
  const double tot = (double)block_sum(acc);
  store_partials(d, tile, &tot, 1);
}

// One workgroup per system and value (grid nsys x nv): sum the generic partials of
// value q in a fixed order into red[red_off + q]; with RED_CG_SETUP the q = 0
// workgroup also starts a CG on rr = result[0]: stop2 = pa + pr*rr, maxit = pi,
// iters 0, active iff rr > stop2.
__global__ __launch_bounds__(kBlock) void k_finish(const SysDesc* __restrict__ sys, LaunchList L, int red_off,
                                                   int mode) {
  const int kk = blockIdx.x, q = blockIdx.y;
  const SysDesc* __restrict__ d = sys + L.sys[kk];
  Scal* sc = d->sc;
  const double s = sum_partials(d->part + q, d->ntiles, kMaxRed);
  if (threadIdx.x == 0) {
    sc->red[red_off + q] = s;
    if (q == 0 && mode == RED_CG_SETUP) {
      const double stop2 = L.pa[kk] + L.pr[kk] * s;
      sc->rrv[0] = s;
      sc->stop2 = stop2;
      sc->maxit = L.pi[kk];
      sc->iters = 0;
      store_active(sc, s > stop2 ? 1 : 0);
    }
  }
}

// Scal records to host-coherent memory, every thread's stores made visible at system
// scope before the barrier, then the flag.
__global__ __launch_bounds__(kBlock) void k_publish(const Scal* __restrict__ d, Scal* h, int nw, unsigned* flag,
                                                    unsigned seq) {
  const unsigned long long* __restrict__ src = reinterpret_cast<const unsigned long long*>(d);
  unsigned long long* dst = reinterpret_cast<unsigned long long*>(h);
  for (int k = threadIdx.x; k < nw; k += kBlock) dst[k] = src[k];
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}


// x = (set ? 0 : x) + sum_{i < cnt} y_i z_i, y from ys (row of the system's slot), z_i the
// C64 slot S_Z0 + i.
template <int SPT>
__global__ __launch_bounds__(kBlock) void k_xupdate(const SysDesc* __restrict__ sys, LaunchList L,
                                                    const double* __restrict__ ys, int cnt, int set) {
  constexpr int TILE = kBlock * SPT;
  HUB_PROLOGUE_T(TILE)
  (void)sc;
  const double* __restrict__ yrow = ys + (size_t)L.sys[kk] * kYStride;
  const Vec<double2> x(d->vec[S_X]);
  double2 xv[SPT];
#pragma unroll
  for (int m = 0; m < SPT; ++m) {
    const int n = base + m * kBlock;
    xv[m] = cz<double2>();
    if (n < t_hi && !set) xv[m] = x[n];
  }
  for (int q = 0; q < cnt; ++q) {
    const double yr = yrow[2 * q], yi = yrow[2 * q + 1];
    const Vec<float2> z(d->vec[S_Z0 + q]);
#pragma unroll
    for (int m = 0; m < SPT; ++m) {
      const int n = base + m * kBlock;
      if (n < t_hi) {
        const float2 zf = z[n];
        const double zr = zf.x, zi = zf.y;
        xv[m].x += yr * zr - yi * zi;
        xv[m].y += yr * zi + yi * zr;
      }
    }
  }
#pragma unroll
  for (int m = 0; m < SPT; ++m) {
    const int n = base + m * kBlock;
    if (n < t_hi) x.set(n, xv[m]);
  }
}

// One Arnoldi step of small systems (at most kArnWgMaxSites sites), one workgroup per
// system: w = (M M^dagger + mu2) z_j in FP64 (the 12-point form), the classical
// Gram-Schmidt coefficients h_i = <v_i, w> against the unmodified w for i <= j, w -= sum_i
// h_i v_i in the order of i, and |w|^2.  Each reduction is a workgroup sum in a fixed order;
// the results land where the tiled path's reductions put them (red[2i], red[2i+1]: h_i,
// red[2(j+1)]: |w|^2).  One launch and one read of the basis replace the tiled path's five
// launches and two reads.
__global__ __launch_bounds__(kWgBlock) void k_arnoldi_wg(const SysDesc* __restrict__ sys, WgList L, int j) {
  const SysDesc* __restrict__ d = sys + L.sys[blockIdx.x];
  Scal* sc = d->sc;
  const Geom g = d->g;
  const int N = g.n;
  const Vec<float2> z(d->vec[S_Z0 + j]);
  const Vec<double2> w(d->vec[S_R]);
  const PhasePhi<double> ph = phase_of<double>(d);
  const double mu2 = d->mu2;
  __shared__ double red[2][kWgBlock / 64];
  auto ld = [=](int k) { return to_c128<float2>(z[k]); };
  __shared__ double hs[2 * (kMaxRestart + 1)];  // the coefficients, for the subtraction pass
#pragma unroll 1
  for (int n = threadIdx.x; n < N; n += kWgBlock) w.set(n, normal12(g, ph, n, mu2, ld));
  // each thread reads back only its own sites of w: no barrier
  double2 w0[kWgPerThread];
#pragma unroll
  for (int m = 0; m < kWgPerThread; ++m) {
    const int n = threadIdx.x + m * kWgBlock;
    w0[m] = cz<double2>();
    if (n < N) w0[m] = w[n];
  }
  int b = 0;
  for (int q = 0; q <= j; ++q) {
    const Vec<double2> v(d->vec[S_V0 + q]);
    double ar = 0.0, ai = 0.0;
#pragma unroll
    for (int m = 0; m < kWgPerThread; ++m) {
      const int n = threadIdx.x + m * kWgBlock;
      if (n < N) {
        const double2 vv = v[n];
        ar += vv.x * w0[m].x + vv.y * w0[m].y;
        ai += vv.x * w0[m].y - vv.y * w0[m].x;
      }
    }
    const double hr = wg_sum(ar, red[b]);
    b ^= 1;
    const double hi = wg_sum(ai, red[b]);
    b ^= 1;
    if (threadIdx.x == 0) {
      hs[2 * q] = hr;
      hs[2 * q + 1] = hi;
      sc->red[2 * q] = hr;
      sc->red[2 * q + 1] = hi;
    }
  }
  __syncthreads();  // hs complete
  // w -= sum_i h_i v_i, in the order of i at every site
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < kWgPerThread; ++m) {
    const int n = threadIdx.x + m * kWgBlock;
    if (n < N) {
      double2 wc = w0[m];
      for (int q = 0; q <= j; ++q) {
        const double2 vv = Vec<double2>(d->vec[S_V0 + q])[n];
        const double hr = hs[2 * q], hi = hs[2 * q + 1];
        wc.x -= hr * vv.x - hi * vv.y;
        wc.y -= hr * vv.y + hi * vv.x;
      }
      w.set(n, wc);
      acc += norm2<double>(wc);
    }
  }
  const double ww = wg_sum(acc, red[b]);
  if (threadIdx.x == 0) sc->red[2 * (j + 1)] = ww;
}

}  // namespace

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
static inline int tiles_of(int n) { return (n + kTile - 1) / kTile; }

template <bool NT>
static void apply_nt(const Geom& g, const double* phi, const double2* x, double2* y, int batch, bool dag,
                     hipStream_t st) {
  const int nt = (g.n + kPubTile - 1) / kPubTile;
  const int per = pub_group(nt, batch);
  const dim3 grid(nt * ((batch + per - 1) / per)), block(kBlock);
  if (per == 1) {
    if (dag)
      hipLaunchKernelGGL((k_apply<true, NT>), grid, block, 0, st, g, phi, x, y, nt);
    else
      hipLaunchKernelGGL((k_apply<false, NT>), grid, block, 0, st, g, phi, x, y, nt);
  } else {
    if (dag)
      hipLaunchKernelGGL((k_apply_grp<true, NT>), grid, block, 0, st, g, phi, x, y, nt, per, batch);
    else
      hipLaunchKernelGGL((k_apply_grp<false, NT>), grid, block, 0, st, g, phi, x, y, nt, per, batch);
  }
}

hipError_t launch_apply(const Geom& g, const double* phi, const double2* x, double2* y, int batch, bool dag,
                        hipStream_t st, bool to_caller) {
  if (to_caller)
    apply_nt<true>(g, phi, x, y, batch, dag, st);
  else
    apply_nt<false>(g, phi, x, y, batch, dag, st);
  return hipGetLastError();
}


hipError_t launch_force(const Geom& g, const double* phi, const double2* eta, const double2* xi, double scale,
                        int accumulate, double* out, int batch, hipStream_t st, const double2* sub) {
  const int nt = tiles_of(g.n);
  // 2048-site tiles: a quarter of the public kernels' workgroups per vector
  const int per = pub_group(4 * nt, batch);
  const dim3 grid(nt * ((batch + per - 1) / per)), block(kBlock);
  if (per == 1)
    hipLaunchKernelGGL(k_force, grid, block, 0, st, g, phi, eta, xi, sub, scale, accumulate, out, nt);
  else
    hipLaunchKernelGGL(k_force_grp, grid, block, 0, st, g, phi, eta, xi, sub, scale, accumulate, out, nt, per,
                       batch);
  return hipGetLastError();
}

hipError_t launch_force_sum(const Geom& g, const double* phi, const double2* eta, const double2* xi,
                            const double* scale_host, int accumulate, double* out, int batch, hipStream_t st) {
  if (batch < 1 || batch > kMaxSys) return hipErrorInvalidValue;
  Mu2Arr sc;
  for (int b = 0; b < kMaxSys; ++b) sc.v[b] = b < batch ? scale_host[b] : 0.0;
  hipLaunchKernelGGL(k_force_sum, dim3(tiles_of(g.n)), dim3(kBlock), 0, st, g, phi, eta, xi, sc, accumulate, out,
                     batch);
  return hipGetLastError();
}

hipError_t launch_stream_bytes(const double* phi, const double2* x, double2* y, int n, int mode, hipStream_t st) {
  const dim3 grid((n + kPubTile - 1) / kPubTile), block(kBlock);
  if (mode == 0)
    hipLaunchKernelGGL((k_stream_bytes<false, true>), grid, block, 0, st, phi, x, y, n);
  else if (mode == 1)
    hipLaunchKernelGGL((k_stream_bytes<true, false>), grid, block, 0, st, phi, x, y, n);
  else
    hipLaunchKernelGGL((k_stream_bytes<false, false>), grid, block, 0, st, phi, x, y, n);
  return hipGetLastError();
}

hipError_t launch_dot_re(const Geom& g, const double2* a, const double2* b, int batch, double* part,
                         double* result, hipStream_t st) {
  const int nt = tiles_of(g.n);
  hipLaunchKernelGGL(k_dot_re, dim3(nt * batch), dim3(kBlock), 0, st, g, a, b, nt, part);
  hipLaunchKernelGGL(k_dot_finish, dim3(batch), dim3(kBlock), 0, st, part, nt, result);
  return hipGetLastError();
}

hipError_t launch_md_drift(double* phi, const double* pi, double eps, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_md_drift, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, phi, pi, eps, n);
  return hipGetLastError();
}

hipError_t launch_md_kick(double* pi, const double* phi, const double* G, double cg, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_md_kick, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, pi, phi, G, cg, n);
  return hipGetLastError();
}

hipError_t launch_ms_start(const MsDesc* d, int ntiles, hipStream_t st) {
  hipLaunchKernelGGL(k_ms_start, dim3(ntiles), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_ms_setup, dim3(1), dim3(kBlock), 0, st, d);
  return hipGetLastError();
}

hipError_t launch_ms_iter(const MsDesc* d, int ntiles, int it, hipStream_t st) {
  hipLaunchKernelGGL(k_ms1, dim3(ntiles), dim3(kBlock), 0, st, d, it);
  hipLaunchKernelGGL(k_ms2, dim3(ntiles), dim3(kBlock), 0, st, d, it);
  return hipGetLastError();
}

hipError_t launch_normal2(const Geom& g, const double* phi, const double mu2_host[kMaxSys], const double2* u,
                          const double2* x, double2* y, int batch, hipStream_t st) {
  const int nt = (g.n + kPubTile - 1) / kPubTile;
  const int per = pub_group(nt, batch);
  Mu2Arr m;
  for (int b = 0; b < kMaxSys; ++b) m.v[b] = b < batch ? mu2_host[b] : 0.0;
  const dim3 grid(nt * ((batch + per - 1) / per)), block(kBlock);
  if (per == 1)
    hipLaunchKernelGGL(k_normal2_pub, grid, block, 0, st, g, phi, m, u, x, y, nt);
  else
    hipLaunchKernelGGL(k_normal2_grp, grid, block, 0, st, g, phi, m, u, x, y, nt, per, batch);
  return hipGetLastError();
}


hipError_t launch_phase(const double* phi, double2* p64, float* p32, int n, hipStream_t st, float2* cs32) {
  hipLaunchKernelGGL(k_phase, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, phi, p64, p32, cs32, n);
  return hipGetLastError();
}

template <int N>
static CgList<N> cg_list(const LaunchList& L) {
  CgList<N> c;
  std::memset(&c, 0, sizeof(c));
  c.scal = L.scal;
  c.nsys = L.nsys;
  c.total_tiles = L.total_tiles;
  for (int k = 0; k <= N; ++k) c.tile_begin[k] = k <= L.nsys ? L.tile_begin[k] : L.total_tiles;
  for (int k = 0; k < L.nsys; ++k) {
    c.sys[k] = L.sys[k];
    c.pi[k] = L.pi[k];
    c.it[k] = L.it[k];
  }
  return c;
}

// One CG stage (1 or 2) over the list; with events, the launch records its own start and end.
template <typename R, int SPT, typename LL>
static void cg_stage(const SysDesc* sys, const LL& c, int stage, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  const dim3 grid(c.total_tiles), block(kBlock);
  const bool single = sizeof(R) == 4;
  const int sR = single ? (int)S_R32 : (int)S_R, sP = single ? (int)S_P32 : (int)S_P0,
            sU = single ? (int)S_U32 : (int)S_U;
  auto kern = stage == 1 ? k_cg1<R, LL, SPT> : k_cg2<R, LL, SPT>;
  if (e0)
    hipExtLaunchKernelGGL(kern, grid, block, 0, st, e0, e1, 0, sys, c, sR, sP, sU);
  else
    hipLaunchKernelGGL(kern, grid, block, 0, st, sys, c, sR, sP, sU);
}

template <typename R, int SPT>
static void cg_stage_list(const SysDesc* sys, const LaunchList& L, int stage, hipStream_t st, hipEvent_t e0,
                          hipEvent_t e1) {
  if (L.nsys <= kSmallCg)
    cg_stage<R, SPT>(sys, cg_list<kSmallCg>(L), stage, st, e0, e1);
  else
    cg_stage<R, SPT>(sys, cg_list<kMaxSys>(L), stage, st, e0, e1);
}

template <typename R>
static void cg_stage_any(const SysDesc* sys, const LaunchList& L, int spt, int stage, hipStream_t st,
                         hipEvent_t e0, hipEvent_t e1) {
  if (spt == kSmallSpt)
    cg_stage_list<R, kSmallSpt>(sys, L, stage, st, e0, e1);
  else
    cg_stage_list<R, kSitesPerThread>(sys, L, stage, st, e0, e1);
}

static bool spt_ok(const LaunchList& L) { return L.spt == kSmallSpt || L.spt == kSitesPerThread; }

hipError_t launch_cg_iter(const SysDesc* sys, const LaunchList& L, bool single, hipStream_t st) {
  if (!spt_ok(L)) return hipErrorInvalidValue;
  for (int stage = 1; stage <= 2; ++stage) {
    if (single)
      cg_stage_any<float>(sys, L, L.spt, stage, st, nullptr, nullptr);
    else
      cg_stage_any<double>(sys, L, L.spt, stage, st, nullptr, nullptr);
  }
  return hipGetLastError();
}

hipError_t launch_cg_stage(const SysDesc* sys, const LaunchList& L, bool single, int stage, hipStream_t st,
                           hipEvent_t e0, hipEvent_t e1) {
  if (!spt_ok(L)) return hipErrorInvalidValue;
  if (single)
    cg_stage_any<float>(sys, L, L.spt, stage, st, e0, e1);
  else
    cg_stage_any<double>(sys, L, L.spt, stage, st, e0, e1);
  return hipGetLastError();
}


hipError_t launch_cg_wg(const SysDesc* sys, const WgList& L, int K, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  // nmax even: the pair path's 16-byte LDS accesses of u stay aligned
  if (L.nsys < 1 || L.nsys > kMaxSys || K < 1 || L.nmax < 2 || L.nmax > kWgMaxSites || (L.nmax & 1))
    return hipErrorInvalidValue;
  // the (cos, sin) tables join p and u in LDS when all three fit
  WgList W = L;
  W.cs_lds = 3 * (size_t)L.nmax * sizeof(float2) <= 2 * (size_t)kWgMaxSites * sizeof(float2) ? 1 : 0;
  const size_t lds = (W.cs_lds ? 3 : 2) * (size_t)L.nmax * sizeof(float2);
  static bool attr_set = false;  // the 160 KB of dynamic LDS exceed the default limit
  if (!attr_set) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_cg_wg32, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)(2 * (size_t)kWgMaxSites * sizeof(float2)));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const dim3 grid(L.nsys), block(kWgBlock);
  if (e0)
    hipExtLaunchKernelGGL(k_cg_wg32, grid, block, lds, st, e0, e1, 0, sys, W, K);
  else
    hipLaunchKernelGGL(k_cg_wg32, grid, block, lds, st, sys, W, K);
  return hipGetLastError();
}

hipError_t launch_arnoldi_wg(const SysDesc* sys, const WgList& L, int j, hipStream_t st) {
  if (L.nsys < 1 || L.nsys > kMaxSys || j < 0 || j >= kMaxRestart || L.nmax > kWgMaxSites) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_arnoldi_wg, dim3(L.nsys), dim3(kWgBlock), 0, st, sys, L, j);
  return hipGetLastError();
}

hipError_t launch_publish(const Scal* d, Scal* h, int cnt, unsigned* flag, unsigned seq, hipStream_t st) {
  if (cnt < 1 || cnt > kMaxSys || !d || !h || !flag) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_publish, dim3(1), dim3(kBlock), 0, st, d, h, cnt * (int)(sizeof(Scal) / 8), flag, seq);
  return hipGetLastError();
}

static hipError_t finish(const SysDesc* sys, const LaunchList& L, int nv, int red_off, RedMode mode,
                         hipStream_t st) {
  if (nv < 1 || nv > kMaxRed || red_off < 0 || red_off + nv > kMaxRed) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_finish, dim3(L.nsys, nv), dim3(kBlock), 0, st, sys, L, red_off, (int)mode);
  return hipGetLastError();
}


// Launch KERNEL<..., SPT> for the tile class of L.
#define HUB_BY_CLASS(KERNEL, GRID, ...)                                                       \
  do {                                                                                       \
    if (L.spt == kSmallSpt)                                                                  \
      hipLaunchKernelGGL(KERNEL<kSmallSpt>, GRID, dim3(kBlock), 0, st, __VA_ARGS__);          \
    else                                                                                     \
      hipLaunchKernelGGL(KERNEL<kSitesPerThread>, GRID, dim3(kBlock), 0, st, __VA_ARGS__);    \
  } while (0)

hipError_t launch_normal_slot(const SysDesc* sys, const LaunchList& L, int s_in, bool in_c64, int s_b, int s_out,
                              RedMode mode, int red_off, hipStream_t st) {
  if (!spt_ok(L)) return hipErrorInvalidValue;
  const dim3 grid(L.total_tiles), block(kBlock);
  const bool small = L.spt == kSmallSpt;
  auto kern = in_c64 ? (small ? k_normal_slot<float2, kSmallSpt> : k_normal_slot<float2, kSitesPerThread>)
                     : (small ? k_normal_slot<double2, kSmallSpt> : k_normal_slot<double2, kSitesPerThread>);
  hipLaunchKernelGGL(kern, grid, block, 0, st, sys, L, s_in, s_b, s_out, (int)mode);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || mode == RED_NONE) return e;
  return finish(sys, L, 1, red_off, mode, st);
}

hipError_t launch_cg_init_zero(const SysDesc* sys, const LaunchList& L, RedMode mode, hipStream_t st) {
  if (!spt_ok(L)) return hipErrorInvalidValue;
  HUB_BY_CLASS(k_cg_init_zero, dim3(L.total_tiles), sys, L);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return finish(sys, L, 1, 0, mode, st);
}

hipError_t launch_multidot(const SysDesc* sys, const LaunchList& L, int s_w, int s_v0, int cnt, int red_off,
                           hipStream_t st) {
  if (!spt_ok(L)) return hipErrorInvalidValue;
  HUB_BY_CLASS(k_multidot, dim3(L.total_tiles), sys, L, s_w, s_v0, cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return finish(sys, L, 2 * cnt, red_off, RED_STORE, st);
}

hipError_t launch_cgs(const SysDesc* sys, const LaunchList& L, int s_w, int s_v0, int cnt, int h_off, int red_off,
                      hipStream_t st) {
  if (!spt_ok(L)) return hipErrorInvalidValue;
  HUB_BY_CLASS(k_cgs, dim3(L.total_tiles), sys, L, s_w, s_v0, cnt, h_off);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return finish(sys, L, 1, red_off, RED_STORE, st);
}

hipError_t launch_prep_inner(const SysDesc* sys, const LaunchList& L, int s_src, int s_v, hipStream_t st) {
  if (!spt_ok(L)) return hipErrorInvalidValue;
  HUB_BY_CLASS(k_prep_inner, dim3(L.total_tiles), sys, L, s_src, s_v);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // only systems that start a single-precision CG (pi > 0) are finalised
  LaunchList F = L;
  int m = 0;
  for (int k = 0; k < L.nsys; ++k)
    if (L.pi[k] > 0) {
      F.sys[m] = L.sys[k];
      F.pa[m] = 0.0;
      F.pr[m] = L.pr[k];
      F.pi[m] = L.pi[k];
      ++m;
    }
  if (m == 0) return hipSuccess;
  F.nsys = m;
  return finish(sys, F, 1, 0, RED_CG_SETUP, st);
}

hipError_t launch_xupdate(const SysDesc* sys, const LaunchList& L, const double* ys, int cnt, bool set,
                          hipStream_t st) {
  if (!spt_ok(L)) return hipErrorInvalidValue;
  HUB_BY_CLASS(k_xupdate, dim3(L.total_tiles), sys, L, ys, cnt, set ? 1 : 0);
  return hipGetLastError();
}

}  // namespace hub
