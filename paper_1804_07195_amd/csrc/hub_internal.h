// Internal types shared by the HIP kernels and the host engine of libhub.
// Not part of the public ABI (see include/hub.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace hub {

constexpr int kBlock = 256;                   // threads per workgroup (4 wave64)
#ifndef HUB_SITES_PER_THREAD
#define HUB_SITES_PER_THREAD 8
#endif
constexpr int kSitesPerThread = HUB_SITES_PER_THREAD;  // sites handled by each thread
constexpr int kTile = kBlock * kSitesPerThread;  // sites per workgroup tile
constexpr int kMaxSys = 64;                   // systems per batched launch
constexpr int kMaxRestart = 20;               // largest FGMRES restart length
constexpr int kMaxRed = 2 * (kMaxRestart + 1) + 2;  // reduced doubles per tile (multi-dot)
constexpr int kNumXcd = 8;                    // accelerator complex dies on MI355X
constexpr int kMaxSlots = 64;                 // vector slots per system

// Exact division by an invariant divisor for 0 <= n < 2^31 (Granlund-Montgomery):
// q = (umulhi(n, m) + n) >> s with s = ceil(log2 d), m = floor(2^32 (2^s - d) / d) + 1.
struct FastDiv {
  uint32_t d, m, s;
};

__host__ __device__ inline uint32_t fdiv(uint32_t n, FastDiv f) {
  uint32_t hi = (uint32_t)(((uint64_t)n * (uint64_t)f.m) >> 32);
  return (hi + n) >> f.s;
}

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t s = 0;
  while ((1ull << s) < d) ++s;
  f.s = s;
  f.m = (uint32_t)(((1ull << 32) * ((1ull << s) - d)) / d + 1);
  return f;
}

// Lattice geometry and couplings of one system, passed by value to kernels.
struct Geom {
  int L1, L2, Nt;
  int P;   // L1*L2 sites per sublattice plane
  int n;   // 2*P*Nt unknowns
  int pad;
  FastDiv dL2, dL1;
  double kappa;  // kappa~ = delta*kappa
  double ms;     // m~ = delta*m_s
};

// Per-system solver state (device memory).  Fields are written by the first
// workgroup of a kernel and read by later kernels only, never by other
// workgroups of the writing kernel (except `active`, whose readers take the same
// decision whichever value they see).
struct Scal {
  double rrv[2];  // |r_k|^2 of CG iteration k in rrv[k & 1]
  double alpha[2];  // alpha_k of CG iteration k in alpha[k & 1]
  double stop2;   // CG stops once |r|^2 <= stop2
  double red[kMaxRed];               // results of the last generic reduction
  int iters;      // CG iterations performed when the CG stopped
  int maxit;
  int active;     // CG: 1 iterating, 2 stopped by the last stage 1 (the next stage 2 sets 0), 0 stopped
  int pad;
};

// Per-system descriptor (device memory, written by the host when a system joins).
struct SysDesc {
  Geom g;
  double mu2;
  const double* phi;     // float64 phi [n]
  const double2* ph64;   // (cos phi, sin phi) [n], FP64 solver kernels
  const float* ph32;     // phi reduced to [-pi, pi] and rounded to float [n] (single-precision path)
  const float2* cs32;    // (cos, sin) of ph32 [n] (single-workgroup CG of small mixed-solver systems)
  Scal* sc;
  double* part;          // per-tile partials of the generic reductions [ntiles][kMaxRed]
  double* part1;         // per-tile partials of CG stage 1 [ntiles]
  double* part2;         // per-tile partials of CG stage 2 [ntiles]
  int ntiles;            // solver tiles (2 Nt tnb), at most kBlock * spt sites each
  int spt;               // sites per thread of every solver kernel of this system (tile class)
  int tnb;               // tiles per segment
  int tbsz;              // sites per tile (the last tile of a segment may hold fewer)
  int tseg;              // sites per segment (a plane, or the whole vector)
  void* vec[kMaxSlots];  // vector slots (type fixed by the slot's role)
};

// Multi-shift CG (FP64): one CG on A_0 = M M^dag + mu2 carrying the shifted systems
// (A_0 + sigma_s) x_s = b through the scalar recurrences of the shared Krylov space.
constexpr int kMsMax = 16;  // shifted systems per solve
struct MsScal {
  double rrv[2];              // |r_k|^2 in rrv[k & 1]
  double alpha[2];            // alpha_k in alpha[k & 1]; alpha[1] = 1 stands for alpha_{-1}
  double beta[2];             // beta_k in beta[k & 1]; beta[1] = 0 stands for beta_{-1}
  double stop2;               // tol^2 |b|^2 (base and shifted residuals)
  double pad0;
  double zeta[kMsMax][3];     // zeta^s_k in zeta[s][k % 3]
  int frozen[kMsMax][2];      // shift s done updating after step k: frozen[s][(k+1) & 1]
  int iters, maxit, active;
  int stop;                   // set by the stage 1 that stops; the next stage 2 clears active
};
struct MsDesc {
  Geom g;
  const double2* ph64;        // (cos phi, sin phi) per site
  double mu2;                 // shift of the base system
  const double2* b;
  double2* x;                 // base solution
  double2* r;
  double2* p[2];
  double2* u;
  double2* xs[kMsMax];        // shifted solutions
  double2* ps[kMsMax];        // shifted search directions
  double sigma[kMsMax];       // mu2_s - mu2 >= 0
  int ns;
  int ntiles;                 // solver tiles (tile_geo with kSitesPerThread)
  int tnb, tbsz, tseg;        // tiles per segment, sites per tile, sites per segment
  double* part1;
  double* part2;
  MsScal* sc;
  double* hist;               // alpha_k at [2k], beta_k at [2k+1] (Lanczos coefficients)
  double tol2;
  int maxit;
  int pad;
};

// Systems of one batched launch: workgroup tiles are laid out system after system.
struct LaunchList {
  Scal* scal;           // the engine's Scal array: system slot k uses scal[k]
  int nsys;
  int total_tiles;
  int spt;              // tile class of every system of the list (sites per thread)
  int pad;
  int tile_begin[kMaxSys + 1];
  int sys[kMaxSys];     // index into the SysDesc array
  double pa[kMaxSys];   // per-system kernel parameters (meaning set by the kernel)
  double pr[kMaxSys];
  int pi[kMaxSys];
  int pj[kMaxSys];
  int it[kMaxSys];      // CG iteration index of each system in this launch
};

// The part of a launch list the CG kernels read, for up to N systems.  It is the
// kernel argument of every CG launch, so it is kept small: N = 4 covers most launches
// (a 2.3 KB argument costs ~0.2 us per launch on the device and more on the host).
template <int N>
struct CgList {
  Scal* scal;
  int nsys;
  int total_tiles;
  int tile_begin[N + 1];
  int sys[N];
  int pi[N];   // solution slot
  int it[N];   // CG iteration index
};
constexpr int kSmallCg = 4;

// Mixed-solver systems of at most kWgMaxSites sites run their complex64 CG in the
// single-workgroup kernel (one workgroup of kWgBlock threads per system, all of its
// state in registers and LDS, a block of iterations per launch); their other solver
// kernels use the small tile class.  The limit: p and u in complex64 (2 x 8 bytes per
// site) plus the reduction scratch fit in the 160 KB of LDS of a gfx950 CU, and a
// thread holds at most kWgPerThread sites.
constexpr int kWgBlock = 1024;
constexpr int kWgPerThread = 10;
#ifndef HUB_WG_MAX_SITES
#define HUB_WG_MAX_SITES 10200
#endif
constexpr int kWgMaxSites = HUB_WG_MAX_SITES;
static_assert(kWgMaxSites <= kWgBlock * kWgPerThread, "sites per thread");
static_assert(kWgPerThread % 2 == 0, "whole site pairs per thread");
static_assert(2 * kWgMaxSites * 8 + 2 * (kWgBlock / 64) * 8 <= 160 * 1024, "LDS of one CU");
inline bool wg_of(int n) { return n <= kWgMaxSites; }
// Systems whose FGMRES Arnoldi step runs as one fused single-workgroup launch instead of
// the tiled kernels: one CU streams the basis twice, which beats the tiled path's launches
// up to about this size (6x6x32: 7% faster per solve, 6x6x64 and 8x8x36: 2-4%, 12x12x32:
// 5% slower).
constexpr int kArnWgMaxSites = 4608;
inline bool arn_wg_of(int n) { return n <= kArnWgMaxSites; }
// Systems of one single-workgroup CG launch: workgroup k runs system sys[k] from
// iteration it[k], solution slot pi[k]; nmax = the largest system (LDS per workgroup).
struct WgList {
  Scal* scal;
  int nsys;
  int nmax;
  int cs_lds;  // set by the launcher: the (cos, sin) tables are staged in LDS (nmax small enough)
  int sys[kMaxSys];
  int pi[kMaxSys];
  int it[kMaxSys];
};

// Tile class of a system: sites per thread of all its solver kernels.  Large systems
// take kSitesPerThread (tiles of at most 2048 sites: fewer workgroups, fixed costs spread
// over more sites); a system below kBigSites takes kSmallSpt (at most 512), so that its grids
// have enough workgroups to hide latency and each thread's serial chain stays short
// (the mixed 102x102x64 step is 15% slower with tiles of at most 1024 sites and 10% slower
// with 4096 than with 2048; a 48x48x64 solve is 5-9% faster and a 12x12x32 one 11-21%
// faster with 512-site tiles than with 1024).  Launch lists hold systems of one class.
#ifndef HUB_SMALL_SPT
#define HUB_SMALL_SPT 2
#endif
constexpr int kSmallSpt = HUB_SMALL_SPT;
constexpr int kBigSites = 300 * kTile;
inline int spt_of(int n) { return n >= kBigSites ? kSitesPerThread : kSmallSpt; }

// Tiles of the batched solver kernels.  The vector is cut into segments of `seg`
// sites, each segment into `nb` tiles of `bsz` sites (the last tile of a segment
// possibly shorter); tile k covers block k % nb of segment k / nb.  A plane (one
// sublattice of one time slice, P = L1*L2 consecutive sites) of at least half a tile
// is a segment of its own, cut into even blocks of at most kBlock*spt sites: a
// site's sublattice partner (one plane away) and its temporal neighbour (two planes
// away) then lie at the same offset of another tile, touched in the same load round
// of that tile, and no tile straddles a plane.  Smaller planes are grouped whole,
// as many as fit in a tile, in one segment spanning the vector.
struct TileGeo {
  int nb, bsz, seg, ntiles;
};
inline TileGeo tile_geo(const Geom& g, int spt) {
  const int T = kBlock * spt, P = g.P;
  TileGeo t;
  if (2 * P >= T) {
    int nb = (P + T - 1) / T;
    int bsz = (P + nb - 1) / nb;
    bsz += bsz & 1;
    nb = (P + bsz - 1) / bsz;  // no empty block after the rounding
    t.nb = nb;
    t.bsz = bsz;
    t.seg = P;
    t.ntiles = 2 * g.Nt * nb;
  } else {
    t.bsz = (T / P) * P;
    t.ntiles = (g.n + t.bsz - 1) / t.bsz;
    t.nb = t.ntiles;
    t.seg = g.n;
  }
  return t;
}

// Vector slot roles.  FP64 slots hold double2 [n]; C64 slots hold float2 [n].
enum Slot : int {
  S_B = 0,     // right-hand side (FP64)
  S_X = 1,     // solution (FP64)
  S_R = 2,     // residual / Arnoldi w (FP64)
  S_P0 = 3,    // CG direction, ping-pong pair S_P0, S_P0+1 (FP64)
  S_U = 5,     // M^dagger p scratch (FP64)
  S_V0 = 6,    // Arnoldi basis v_0 .. v_m (FP64), up to S_V0 + kMaxRestart
  S_R32 = 40,  // single-precision CG residual (C64)
  S_P32 = 41,  // single-precision CG direction pair S_P32, S_P32+1 (C64)
  S_U32 = 43,  // single-precision M^dagger p scratch (C64)
  S_Z0 = 44    // preconditioned directions z_0 .. z_{m-1} (C64), up to S_Z0 + kMaxRestart - 1
};
static_assert(S_V0 + kMaxRestart < S_R32, "slot layout");
static_assert(S_Z0 + kMaxRestart <= kMaxSlots, "slot layout");

// What a reduction finalisation does with its sums.
enum RedMode : int {
  RED_NONE = 0,
  RED_STORE = 1,     // sc->red[off..] = results
  RED_CG_SETUP = 2   // also CG (re)start: rrv[0] = result[0], stop2 = pa + pr*rr, iters 0, active
};

// ---------------------------------------------------------------------------
// Kernel launchers (hub_kernels.hip).  All enqueue on `st` and return the HIP error.
// ---------------------------------------------------------------------------
// y_b = M x_b or M^dagger x_b.  to_caller: y is the caller's result (stored
// non-temporally); otherwise library workspace that a following kernel reads.
hipError_t launch_apply(const Geom& g, const double* phi, const double2* x, double2* y, int batch,
                        bool dag, hipStream_t st, bool to_caller = false);
// out (+)= scale dS/dphi for eta and xi (minus `sub` when given: Hasenbusch ratio terms).
hipError_t launch_force(const Geom& g, const double* phi, const double2* eta, const double2* xi,
                        double scale, int accumulate, double* out, int batch, hipStream_t st,
                        const double2* sub = nullptr);
// Measurement: a streaming kernel moving the bytes of one FP64 apply of n sites (mode 0:
// non-temporal stores, 1: non-temporal loads, 2: plain).
hipError_t launch_stream_bytes(const double* phi, const double2* x, double2* y, int n, int mode, hipStream_t st);
// out (+)= sum_b scale_host[b] dS_b/dphi over a batch of eta, xi (out: one field of N).
hipError_t launch_force_sum(const Geom& g, const double* phi, const double2* eta, const double2* xi,
                            const double* scale_host, int accumulate, double* out, int batch, hipStream_t st);
hipError_t launch_dot_re(const Geom& g, const double2* a, const double2* b, int batch, double* part,
                         double* result, hipStream_t st);
// p64 = (cos phi, sin phi) in FP64 and, if p32 is not NULL, phi reduced to [-pi, pi]
// and rounded to float (the complex64 kernels evaluate the phase from it).
// With cs32, also (cos, sin) of that float angle as the complex64 kernels evaluate it (the
// single-workgroup CG reads it instead of evaluating it twice per site and iteration).
hipError_t launch_phase(const double* phi, double2* p64, float* p32, int n, hipStream_t st,
                        float2* cs32 = nullptr);
// y_b = M u_b + mu2_b x_b (the second pass of the public normal operator, u = M^dagger x).
hipError_t launch_normal2(const Geom& g, const double* phi, const double mu2_host[kMaxSys], const double2* u,
                          const double2* x, double2* y, int batch, hipStream_t st);
// phi += eps pi;  pi -= G + cg phi (G may be NULL).
hipError_t launch_md_drift(double* phi, const double* pi, double eps, int n, hipStream_t st);
hipError_t launch_md_kick(double* pi, const double* phi, const double* G, double cg, int n, hipStream_t st);

// Batched solver kernels over the systems of a LaunchList (descriptors in `sys`).
// FP64 or C64 CG iteration in two stages (see hub_kernels.hip).
// The batched solver launchers below take systems of one tile class (L.spt).
// Copy the Scal records d[0, cnt) to host-coherent memory h[0, cnt), then write seq to
// *flag (host-coherent) with a system-scope release, so that the host can poll the
// flag instead of synchronising the stream.  One workgroup.
static_assert(sizeof(Scal) % 8 == 0, "Scal is copied in 8-byte words");
hipError_t launch_publish(const Scal* d, Scal* h, int cnt, unsigned* flag, unsigned seq, hipStream_t st);
hipError_t launch_cg_iter(const SysDesc* sys, const LaunchList& L, bool single, hipStream_t st);
// One stage (1 or 2) of the CG iteration.  With events, the launch records the
// kernel's own start and end timestamps into them (hipExtLaunchKernel).
hipError_t launch_cg_stage(const SysDesc* sys, const LaunchList& L, bool single, int stage, hipStream_t st,
                           hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
// K iterations of the complex64 CG of every system of L, one workgroup per system
// (small systems, see kWgMaxSites); optional start/stop events.
hipError_t launch_cg_wg(const SysDesc* sys, const WgList& L, int K, hipStream_t st,
                        hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
// Arnoldi step j (w = A z_j, Gram-Schmidt against v_0 .. v_j, |w|^2 into the Scal records)
// of every system of L, one workgroup per system (small systems, see kArnWgMaxSites).
hipError_t launch_arnoldi_wg(const SysDesc* sys, const WgList& L, int j, hipStream_t st);
// Multi-shift CG: start (r = b, x = 0, x_s = 0, p_s = b, partial |b|^2), setup (one
// workgroup: scalars), and the two stages of iteration `it` (shifted updates of step
// it-1 ride in stage 1, where beta_{it-1} is known).
hipError_t launch_ms_start(const MsDesc* d, int ntiles, hipStream_t st);
hipError_t launch_ms_iter(const MsDesc* d, int ntiles, int it, hipStream_t st);
// Algorithmic bytes per site of each CG stage (reads + writes of distinct vectors).
// FP64 reads the phase e^{i phi} precomputed (16 bytes per site); complex64 reads the
// reduced angle as a float (4 bytes) and evaluates cos and sin in registers.  Stage 2
// updates the solution at odd iterations only (x and p_{it-1} read, x written).
constexpr double kCgBytes[2][3] = {{80.0, 80.0, 128.0}, {36.0, 36.0, 60.0}};  // [single][stage 1, 2 even, 2 odd]
inline double cg_bytes(bool single, int stage, int it) {
  return kCgBytes[single ? 1 : 0][stage == 1 ? 0 : 1 + (it & 1)];
}
// Every reduction below leaves per-tile partials; a finalisation kernel (one
// workgroup per system and value) sums them in a fixed order into sc->red[red_off..] and,
// with RED_CG_SETUP, starts a CG on the result (pa, pr, pi of the launch list).
// out = [b -] (M M^dagger + mu2) in, in one pass of the 12-point form (in: an FP64
// slot or, with in_c64, a complex64 slot), |out|^2 (mode RED_NONE: no reduction).
hipError_t launch_normal_slot(const SysDesc* sys, const LaunchList& L, int s_in, bool in_c64, int s_b, int s_out,
                              RedMode mode, int red_off, hipStream_t st);
// x = 0, r = b, |b|^2 -> red[0]; with RED_CG_SETUP also the FP64 CG start.
hipError_t launch_cg_init_zero(const SysDesc* sys, const LaunchList& L, RedMode mode, hipStream_t st);
// red[off + 2i, 2i+1] = <v_i, w>, i < cnt.
hipError_t launch_multidot(const SysDesc* sys, const LaunchList& L, int s_w, int s_v0, int cnt, int red_off,
                           hipStream_t st);
// w -= sum_i h_i v_i with h = red[h_off..]; |w|^2 -> red[red_off].
hipError_t launch_cgs(const SysDesc* sys, const LaunchList& L, int s_w, int s_v0, int cnt, int h_off,
                      int red_off, hipStream_t st);
// v = pa*src (FP64, stored if s_v >= 0) and the single-precision CG start on it:
// pi = maxit > 0: r32 = c64(v), z = 0, |r32|^2 -> setup with stop2 = pr*rr;
// pi = 0 (no preconditioning): z = c64(v).  z is the slot pj.
hipError_t launch_prep_inner(const SysDesc* sys, const LaunchList& L, int s_src, int s_v, hipStream_t st);
// x = (set ? 0 : x) + sum_{i<cnt} y_i z_i, z the C64 slots from S_Z0 and y of the system in
// slot k at ys + k * kYStride (re, im interleaved).
constexpr int kYStride = 2 * kMaxRestart;
hipError_t launch_xupdate(const SysDesc* sys, const LaunchList& L, const double* ys, int cnt, bool set,
                          hipStream_t st);

}  // namespace hub
