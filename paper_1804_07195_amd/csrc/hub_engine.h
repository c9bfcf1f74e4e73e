// Host side of libhub: workspace pool and the batched solver engine.
#pragma once

#include <complex>
#include <cstdint>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "hub.h"
#include "hub_internal.h"

namespace hub {

// Thread-local error message behind hub_last_error().
void set_error(const std::string& msg);
const char* get_error();

// Stream-ordered caching allocator of device memory, bounded by a byte budget.
// A freed block is reused by the same stream at once and by other streams once
// the work enqueued before its release has finished.
class Pool {
 public:
  Pool(int device, size_t budget);
  ~Pool();
  // Returns nullptr (and sets the error) when the budget would be exceeded.
  void* alloc(size_t bytes, hipStream_t st);
  void release(void* p, hipStream_t st);
  // Release several blocks after the same stream work: one event orders all of them.
  void release_all(const std::vector<void*>& ps, hipStream_t st);
  size_t budget() const { return budget_; }
  size_t in_use() const;
  size_t reserved() const;
  // Bytes a request of this size takes from the budget (granularity rounding).
  static size_t rounded(size_t bytes);

 private:
  // An event recorded after the work that used a group of released blocks, destroyed
  // when the last block of the group is handed out again or freed.
  struct SharedEvent {
    hipEvent_t ev = nullptr;
    int refs = 0;
  };
  struct Block {
    void* p;
    size_t bytes;
    hipStream_t st;
    SharedEvent* ev;
  };
  void drop_event(SharedEvent* e, bool wait);
  int device_;
  size_t budget_;
  size_t reserved_ = 0;  // bytes obtained from hipMalloc
  size_t used_ = 0;      // bytes handed out
  std::vector<Block> free_;
  std::vector<std::pair<void*, size_t>> live_;
  mutable std::mutex mu_;
};

// Block length (CG iterations between flag reads) near a system's expected end.
constexpr int kTailBlock = 4;
// Block length when only single-workgroup systems iterate (their kernel leaves the
// block at convergence).
constexpr int kWgBlockIters = 48;

// Host-side state of one linear system (M M^dagger + mu2) x = b.
struct System {
  // inputs
  Geom g;
  double mu2 = 0.0;
  const double* phi = nullptr;
  const double2* ph64 = nullptr;  // (cos phi, sin phi); computed on add if NULL
  const float* ph32 = nullptr;    // reduced float phi (mixed solver); computed on add if NULL
  const float2* cs32 = nullptr;   // (cos, sin) of ph32 (small mixed-solver systems); computed on add if NULL
  const double2* b = nullptr;
  double2* x = nullptr;
  hub_solve_opts opts{};
  // outputs
  hub_solve_info info{};
  hub_status status = HUB_OK;
  bool done = false;
  // engine bookkeeping
  int slot = -1;
  int phase = 0;
  int post = 0;         // what follows the running single-precision CG
  int j = 0;            // Arnoldi step
  int cycles = 0;
  int cg_total = 0;     // FP64 CG iterations over all restarts
  int enq = 0;          // CG iterations enqueued since the last CG setup
  int gen = 0;          // number of CG setups so far (tags in-flight blocks)
  int pred = 0;         // iterations of the system's previous CG run (0: none yet)
  bool wg = false;      // CG iterations in the single-workgroup kernel (small systems)
  double bnorm = 0.0, err = 0.0, wnorm = 0.0, rnorm_cycle = 0.0, bb = -1.0;
  std::vector<std::complex<double>> H;  // (m+1) x m, column-major
  std::vector<void*> owned;             // workspace blocks of this system
  SysDesc desc{};
  std::function<void(System*)> on_done; // serving: S, force and completion
  void* user = nullptr;
};

// Drives any number (<= kMaxSys) of systems of any lattice sizes to convergence on
// one stream.  Systems iterate together: every CG iteration is one pair of launches
// over all systems currently iterating, whatever their phase or shape.
class Engine {
 public:
  Engine(Pool* pool, hipStream_t st);
  ~Engine();
  // False if the engine's own device or pinned buffers could not be allocated.
  bool ok() const { return ok_; }
  // Allocate workspace and join.  ADD_NO_ROOM (with the error set): no free slot or
  // the workspace is over budget; ADD_HIP: a HIP call failed while joining.
  enum AddResult { ADD_OK = 0, ADD_NO_ROOM = 1, ADD_HIP = 2 };
  AddResult add(System* s);
  // Remove a finished system and return its workspace to the pool.
  void remove(System* s);
  // Advance every system: host-side phases, then one block of CG iterations.
  // Returns the HIP error if any.
  hipError_t step();
  bool idle() const;
  int count() const;
  hipStream_t stream() const { return st_; }
  // Workspace bytes a system of this shape and solver needs.
  static size_t workspace_bytes(const Geom& g, const hub_solve_opts& o);
  // Kernel timing of the CG stages (HIP events around every launch).
  struct KernelStat {
    int64_t launches = 0;
    double ms = 0.0;
    double bytes = 0.0;
  };
  void set_profiling(bool on);
  // [single][kernel]: stage 1, stage 2 of the tiled CG; the single-workgroup CG block
  KernelStat stat[2][3];
  // Serving epilogue of a converged system: S = Re chi^dagger x (host), and
  // dS/dphi into dSdphi (device, may be null).  Synchronises the stream.
  hipError_t finalize(System* s, const double2* chi, double* dSdphi, double* S);

 private:
  // One host-side transition of a group of systems at the same phase.
  hipError_t group_phase(int phase, const std::vector<System*>& g);
  // FP64 CG: the true residual of the iterates of g; restart or stop each system.
  hipError_t confirm(const std::vector<System*>& g);
  // A block of CG iterations enqueued for the systems of one precision, whose
  // convergence flags are read back asynchronously.
  struct Block {
    bool single = false;
    int k = 0;
    int buf = 0;
    std::vector<System*> v;             // grouped by tile class, then the single-workgroup systems
    std::vector<int> cls_end;           // end of each tile class in v
    int nwg = 0;                        // single-workgroup systems at the end of v
    std::vector<hipEvent_t> wgev;       // start/stop of their launch (profiling)
    std::vector<int> gen;               // System::gen of each system at enqueue
    std::vector<std::vector<int>> its;  // iteration index per launch and system (profiling)
    std::vector<hipEvent_t> kev;        // kernel start/stop events (profiling)
    unsigned seq = 0;                   // the block's flags are home once *h_blk_flag_ reaches seq
  };
  hipError_t launch_block(bool single, bool& launched);
  hipError_t finish_block(Block& b);
  hipError_t wait_block(unsigned seq);
  hipError_t read_scal(const std::vector<System*>& v);
  // Descriptors and FGMRES update coefficients go to pinned staging rows (slot-indexed)
  // and reach the device in one copy per kind: flush_desc at the start of every step,
  // flush_y before the update kernel.  A row is rewritten only after the kernels that
  // read its last copy have been waited for.
  void upload_desc(System* s);
  void upload_y(System* s, const std::vector<std::complex<double>>& y);
  hipError_t flush_desc();
  hipError_t flush_y();
  LaunchList one(System* s) const;
  // Launch list over v (systems of one tile class).
  LaunchList list(const std::vector<System*>& v) const;
  void finish(System* s, hub_status st);

  Pool* pool_;
  hipStream_t st_;
  bool ok_ = false;
  SysDesc* d_desc_ = nullptr;
  SysDesc* h_desc_ = nullptr;   // pinned staging of d_desc_
  double* d_y_ = nullptr;       // update coefficients, kYStride doubles per slot
  double* h_y_ = nullptr;       // pinned staging of d_y_
  int desc_lo_ = kMaxSys, desc_hi_ = -1, y_lo_ = kMaxSys, y_hi_ = -1;  // rows to copy
  Scal* d_scal_ = nullptr;
  Scal* h_scal_ = nullptr;      // pinned mirror
  Scal* h_pub_ = nullptr;       // host-coherent copy written by k_publish, followed by its flag
  unsigned* h_pub_flag_ = nullptr;
  unsigned pub_seq_ = 0;
  std::vector<System*> slots_;
  bool profiling_ = false;
  std::vector<hipEvent_t> events_;      // pool for kernel timing
  std::vector<Block> inflight_[2];      // per precision, oldest first
  Scal* h_flags_ = nullptr;             // host-coherent, 4 buffers x kMaxSys, then h_blk_flag_
  unsigned* h_blk_flag_ = nullptr;      // sequence number of the last block whose flags were written
  unsigned blk_seq_ = 0;
  int next_buf_[2] = {0, 0};
};

// y = argmin |beta e_1 - H y| for the (k+1) x k upper Hessenberg H (column-major, leading
// dimension ldh), by Givens rotations; *resid (if not NULL) receives the minimal residual.
std::vector<std::complex<double>> hessenberg_lsq(const std::vector<std::complex<double>>& H, int ldh, int k,
                                                 double beta, double* resid = nullptr);

Geom make_geom(const hub_lattice& lat);
int ntiles_of(int n);

}  // namespace hub
