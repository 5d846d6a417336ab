// Internal declarations shared by the HIP sources of libmbl.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/mbl.h"

namespace mbl {

constexpr int kMaxL = 32;
constexpr int kPascal = kMaxL + 1;  // C(i, t) for 0 <= i, t <= 32

// Internal failure carrying the ABI status; caught at the C boundary.
struct Error : std::runtime_error {
  mbl_status status;
  Error(mbl_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

[[noreturn]] inline void fail(mbl_status s, const std::string& m) { throw Error(s, m); }

#define MBL_HIP(call)                                                             \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      ::mbl::fail(e_ == hipErrorOutOfMemory ? MBL_ENOMEM : MBL_EDEVICE,           \
                  std::string(#call) + ": " + hipGetErrorString(e_));             \
  } while (0)

#define MBL_CHECK_LAUNCH() MBL_HIP(hipGetLastError())

// Device allocation through the installed callback, else hipMallocAsync on
// the stream (`ordered`: work buffers, freed stream-ordered so concurrent
// solves never wait on a device-wide free) or hipMalloc (long-lived tables).
// The allocator that served a buffer is recorded with it and frees it, so a
// callback installed or removed in between never sees foreign pointers.
struct AllocOwner {
  mbl_free_fn free_fn = nullptr;  // callback that frees it, or nullptr (HIP)
  void* ctx = nullptr;
  bool ordered = true;            // HIP path: hipFreeAsync (else hipFree)
  hipStream_t s = nullptr;        // stream handed to the free
};
void* dev_alloc(size_t bytes, hipStream_t s, bool ordered, AllocOwner* owner);
void dev_free(void* p, const AllocOwner& owner);

// Owning device buffer.
class DevBuf {
 public:
  DevBuf() = default;
  DevBuf(size_t bytes, hipStream_t s) { reset(bytes, s); }
  ~DevBuf() { release(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p_(o.p_), n_(o.n_), own_(o.own_) {
    o.p_ = nullptr;
    o.n_ = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p_ = o.p_; n_ = o.n_; own_ = o.own_;
      o.p_ = nullptr; o.n_ = 0;
    }
    return *this;
  }
  // stream-ordered work buffer, freed on the same stream
  void reset(size_t bytes, hipStream_t s) { alloc(bytes, s, true); }
  // long-lived buffer (outlives the stream it was made on): hipMalloc/hipFree
  void reset_persistent(size_t bytes) { alloc(bytes, nullptr, false); }
  // stream-ordered buffer freed on stream `release_on` (which must outlive it)
  void reset_ordered(size_t bytes, hipStream_t s, hipStream_t release_on) {
    alloc(bytes, s, true);
    own_.s = release_on;
  }
  void release() {
    if (p_) dev_free(p_, own_);
    p_ = nullptr;
    n_ = 0;
  }
  template <class T> T* as() const { return static_cast<T*>(p_); }
  void* get() const { return p_; }
  size_t bytes() const { return n_; }

 private:
  void alloc(size_t bytes, hipStream_t s, bool ordered) {
    release();
    if (bytes) p_ = dev_alloc(bytes, s, ordered, &own_);
    n_ = bytes;
  }
  void* p_ = nullptr;
  size_t n_ = 0;
  AllocOwner own_;
};

// One tile of the two-pass (split) apply.  The chain is cut between sites q-1
// and q; a state is s = (hi << q) | lo.  In row order (ascending s) the rows
// with one fixed hi form a contiguous block, indexed by the colex rank of lo
// among the q-site configurations with the same number of up spins.
//   low pass : tile = one block (fixed hi); row0 = first row, code = hi,
//              aux = index of the block's first lo configuration in lo_states.
//   high pass: tile = one lo configuration and every hi it combines with;
//              row0 = colex rank j of lo, code = lo, aux = index of the first
//              hi configuration in hi_states / hoff.
// code and the *_info tables pack a configuration as value | (nd << 24), nd
// being its number of anti-aligned bonds inside the half.  E is the energy of
// the half (ZZ of its inner bonds and its fields); for the tile it is the
// energy of the fixed half (code).
// Low pass only: the rows whose middle bond (q-1, q) is anti-aligned are
// u >= msplit (hi even) or u < msplit (hi odd), msplit = C(q-1, k_lo), and their
// flip targets are the consecutive rows mbase + u of the block hi ^ 1.
struct SplitTile {
  int32_t row0;
  int32_t nrows;
  uint32_t code;
  int32_t aux;
  double E;
  int32_t mbase;
  int32_t msplit;
};

// Tables of the split apply, built once per sector (sizes 2^q and 2^(L-q)).
struct SplitTables {
  bool ok = false;
  int q = 0, Lh = 0;
  int maxrows[2] = {0, 0};       // largest tile of the low [0] / high [1] pass
  int maxmid = 0;                // most middle-bond rows of one low-pass tile
  int ntiles[2] = {0, 0};
  int xcd_first[2][9] = {};      // per pass: tiles [xcd_first[x], xcd_first[x+1]) go to XCD x
  DevBuf tiles[2];               // SplitTile lists of the two passes
  DevBuf lo_info, hi_info;       // uint32: configurations sorted by (up spins, value), packed
  DevBuf lo_E, hi_E;             // double, parallel to lo_info / hi_info
  DevBuf hoff;                   // uint32, parallel to hi_info: first row of that hi's block
  DevBuf Elo_v, Ehi_v;           // double by value (for the diagonal kernel)
};

// Per-sector Hamiltonian data (the opaque mbl_ham).
struct Ham {
  int L = 0, nup = 0;
  int64_t n = 0;
  double J = 1, Delta = 1;
  double h[kMaxL] = {};
  double hsum = 0;
  DevBuf pascal;   // uint32 C[33][33]
  DevBuf states;   // uint32 [n]
  DevBuf diag;     // double [n]  <s|H|s>
  std::vector<uint32_t> pascal_host;
  SplitTables split;
  // Stream the tables are allocated and freed on, stream-ordered (worker
  // solves of the batch and the server), or nullptr: hipMalloc / hipFree
  // after a device synchronisation (handles of the C ABI).
  hipStream_t home = nullptr;
  void table(DevBuf& d, size_t bytes, hipStream_t s) const {
    if (home)
      d.reset_ordered(bytes, s, home);
    else
      d.reset_persistent(bytes);
  }
};

// Host Pascal table C[i][t] (row-major, 33 x 33), 0 where t > i.
std::vector<uint32_t> pascal_table();

// ---- kernels shared between translation units ------------------------------

// Device-side column state of the block PCG (per column j).
struct PcgCoef {
  double rho, pap, alpha, beta;
  int live;
  int pad;
};

// Block CG vectors of one column chunk (w columns) for the split CG steps.
template <class T>
struct SplitCg {
  T* x;
  int64_t ldx;
  T* r;
  int64_t ldr;
  T* p;
  int64_t ldp;
  T* t;
  int64_t ldt;
  const PcgCoef* coef;
  double* part;
  int w;
};
// The chunk can run the split CG steps (usable path, 16-byte aligned vectors).
template <class T>
bool split_cg_ready(const Ham& H, const SplitCg<T>& c);
// Enqueues one fused CG apply through the two passes.
//   op 0: p = M^-1 r + beta p (live columns), t = (H - sigma) p, |t|^2 partials
//   op 1: r -= alpha (H - sigma) t, x += alpha p, r.M^-1 r partials (x in the
//         first pass)
// Partials go to c.part as [column][workgroup]; returns the workgroup count
// per column for the fold kernel.
template <class T>
int split_cg_apply(const Ham& H, double sigma, int op, const SplitCg<T>& c, hipStream_t s);

// Apply launcher: Y = (H - sigma) X over columns [0, w).
template <class T>
void launch_apply(const Ham& H, double sigma, const T* X, int64_t ldx, T* Y, int64_t ldy, int w,
                  hipStream_t s);

// Split (two-pass) apply, an alternative to the one-pass kernel selected with
// MBL_APPLY_SPLIT=1.  split_usable: switched on, the sector has split tables and
// a launch plan exists for rows of row_bytes (whole 16-byte vectors).
// split_apply enqueues Y = (H - sigma) X, or returns false, enqueuing nothing,
// when the path is off or the pointers / strides are not 16-byte aligned.
bool split_usable(const Ham& H, int row_bytes);
template <class T>
bool split_apply(const Ham& H, double sigma, const T* X, int64_t ldx, T* Y, int64_t ldy, int w,
                 hipStream_t s);
// Builds H.split (host tables, uploaded with stream s).
void build_split_tables(Ham& H, hipStream_t s);

// Optional HIP-event timing of the two fused CG apply kernels.
struct PcgTiming {
  static constexpr int kSample = 64;  // timed CG steps per inner solve
  hipEvent_t ev[4 * kSample] = {};
  bool ready = false;
  int64_t launches[2] = {0, 0};
  double ms[2] = {0, 0};
  double bytes[2] = {0, 0};  // algorithmic bytes of the timed launches
  // Every CG step run (the timed ones included): launches, algorithmic
  // bytes, and device time estimated per CG call as its timed sample's mean
  // times the steps that call ran (the untimed steps replay the same launches).
  int64_t launches_all = 0;
  double ms_all[2] = {0, 0};
  double bytes_all[2] = {0, 0};
  bool split = false;        // the timed steps ran the two-pass kernels
  void init();
  ~PcgTiming();
};

// Optional HIP-event timing of a solve's phases (mbl_solve_opts.timing):
// plain applies, Gram products and the small dense kernels.  A solve installs
// its clock for its own thread (t_phase_clock); the launchers of those kernels
// bracket their launches with a PhaseTick, which does nothing when no clock is
// installed.  collect() harvests finished pairs after a stream sync.
struct PhaseClock {
  enum { APPLY = 0, GRAM = 1, SMALL = 2 };
  double ms[3] = {0, 0, 0};
  struct Pair {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Pair> pend;
  std::vector<hipEvent_t> pool;
  hipEvent_t get();
  void collect();
  ~PhaseClock();
};
extern thread_local PhaseClock* t_phase_clock;
struct PhaseTick {
  PhaseClock* c = nullptr;
  int kind = 0;
  hipEvent_t a = nullptr;
  hipStream_t s = nullptr;
  PhaseTick(int k, hipStream_t st);
  ~PhaseTick();
  PhaseTick(const PhaseTick&) = delete;
  PhaseTick& operator=(const PhaseTick&) = delete;
};

// When a solve must stop early: a wall-clock deadline and/or a flag another
// thread sets.  Checked between outer iterations and between chunks of
// replayed CG steps.
struct StopCheck {
  bool has_deadline = false;
  std::chrono::steady_clock::time_point deadline{};
  const volatile int* flag = nullptr;
  bool triggered() const {
    if (flag && *flag != 0) return true;
    return has_deadline && std::chrono::steady_clock::now() >= deadline;
  }
};

// PCG: W = PCG_m(R) (columns independent) with Jacobi diagonal jac.  The
// leading `keep` columns run max(m, m_keep) steps, the others m (keep < 0: all
// run m).  With a stop check, fewer steps may run (W is then the CG iterate
// reached).
template <class T>
void run_pcg(const Ham& H, double sigma, const T* jac, const T* R, int64_t ldr, T* W, int64_t ldw,
             int b, int m, hipStream_t s, PcgTiming* tm = nullptr,
             const StopCheck* stop = nullptr, int keep = -1, int m_keep = 0);

// Fused CG of concurrent solves (the batch): while a thread's t_cg_fuser is
// set, its run_pcg calls without a stop check, timing or guard columns join
// the other threads' calls with the same launch plan in one launch per
// kernel; each problem keeps the bits of its own launch.  max_group <= 8;
// wait_ms: how long the first caller of a group waits for the others.
struct CgFuser;
CgFuser* cg_fuser_create(int max_group, double wait_ms);
void cg_fuser_destroy(CgFuser* f);
void cg_fuser_stats(const CgFuser* f, int64_t* groups, int64_t* jobs);
extern thread_local CgFuser* t_cg_fuser;

// Jacobi diagonal of the fold, d = (E - sigma)^2 + (J/2)^2 * (#active bonds).
template <class T>
void launch_jacobi(const Ham& H, double sigma, T* out, hipStream_t s);

// Gram C = A^T B (FP64 p x q, row-major ldc) with deterministic reduction.
template <class T>
void launch_gram(int64_t n, const T* A, int64_t lda, int p, const T* B, int64_t ldb, int q,
                 double* C, int64_t ldc, hipStream_t s);

// Launch plan of the Gram: tiles x splits workgroups, each split's FP64
// partial p x q tile in `part` (part_bytes).  The plan depends only on
// (n, p, q, same operand), so every caller sums in the same order.
struct GramPlan {
  int sym = 0, tiles = 0;
  int64_t splits = 0, rows = 0;
  size_t part_bytes = 0;
};
GramPlan gram_plan(int64_t n, int p, int q, bool same_operand);
template <class T>
void launch_gram_part(const GramPlan& g, int64_t n, const T* A, int64_t lda, int p, const T* B,
                      int64_t ldb, int q, double* C, int64_t ldc, double* part, hipStream_t s);
// Device address of the fixed Gram scratch (kGramScratchBytes) on the current
// device; looked up once per device.
constexpr size_t kGramScratchBytes = MBL_GRAM_SCRATCH_BYTES;
double* gram_scratch();

// Y = A C (+ beta Y), C FP64 (p x q).
template <class T>
void launch_combine(int64_t n, const T* A, int64_t lda, int p, const double* C, int64_t ldc, T* Y,
                    int64_t ldy, int q, double beta, hipStream_t s);

// Small dense (single workgroup) FP64 kernels; matrices row-major.
// small_eigh: ascending eigenvalues w and eigenvectors V (columns) of the
// symmetric A; V == nullptr asks for eigenvalues only (m <= 128).
void small_eigh(int m, const double* A, int64_t lda, double* w, double* V, int64_t ldv,
                double* work, hipStream_t s);

// Workspace bytes needed by small_eigh for size m.
size_t small_eigh_work_bytes(int m);

template <class S, class D>
void launch_convert(int64_t n, int b, const S* X, int64_t ldx, D* Y, int64_t ldy, hipStream_t s);
void launch_diag_precond(int64_t n, int b, const double* R, int64_t ldr, const double* E,
                         double sign, const double* mu, double floor, double* W, int64_t ldw,
                         hipStream_t s);
template <class T>
void launch_randn(int64_t n, int b, uint64_t seed, T* X, int64_t ldx, hipStream_t s);

// Builds the Pascal table, state list and diagonal of H (device).
void build_tables(Ham& H, hipStream_t s);
// Row index of each 64-bit state (device arrays), -1 if not in the sector.
void rank_states(const Ham& H, const uint64_t* q_dev, int64_t cnt, int64_t* out_dev,
                 hipStream_t s);

mbl_status solve_interior(const Ham& H, double sigma, int nev, int b, double tol,
                          const mbl_solve_opts& o, double* evals, double* evecs, int64_t ldv,
                          double* resid, mbl_solve_info* info, hipStream_t s);
mbl_status spectrum_bounds(const Ham& H, double tol, double* emin, double* emax, hipStream_t s);

// Validated construction of a sector handle (throws Error on bad input);
// home: see Ham::home.
Ham* create_ham(int L, double Sz, double J, double Delta, const double* h_host, hipStream_t s,
                hipStream_t home = nullptr);
// Sector dimension C(L, Sz + L/2) (throws Error for a sector that does not exist).
int64_t sector_dim(int L, double Sz);

// Independent solves (service.hip).
size_t solve_footprint(int L, double Sz, int b, int prec);
mbl_status batch_solve(int count, const mbl_problem* probs, mbl_result* res, int conc);
struct Server;
mbl_status server_create(int device, int conc, size_t budget, Server** out);
mbl_status server_cancel(Server* srv, uint64_t ticket);
mbl_status server_submit(Server* srv, const mbl_problem* rq, uint64_t* ticket);
mbl_status server_wait(Server* srv, uint64_t ticket, double timeout_s, mbl_result* out);
mbl_status server_stats(Server* srv, mbl_server_stats* st);
void server_destroy(Server* srv);

// Observables and spectrum slices (observables.hip).
void entanglement_entropy(const Ham& H, const double* V, int64_t ldv, int nev, int cut, double* S,
                          hipStream_t s);
double mean_gap_ratio(const double* e, int count);
mbl_status solve_slices(const Ham& H, int count, const double* sigmas, int nev, int b, double tol,
                        const mbl_solve_opts& o, double* evals, double* resid, int conc);

}  // namespace mbl
