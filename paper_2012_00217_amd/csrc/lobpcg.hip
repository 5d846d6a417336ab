// LOBPCG on the spectral fold (H - sigma I)^2 with a Jacobi-PCG
// preconditioner (paper Sec. 3.2), and on +-H for the spectrum bounds.
//
// Iteration (orthonormal-basis form; the paper defers the LOBPCG details to
// its references, these choices are standard):
//   S = [X | P | W], kept orthonormal: X, P orthonormal and mutually
//   orthogonal; W = PCG_m(A X - X mu) is orthogonalised against [X P] twice and
//   orthonormalised by Cholesky-QR applied twice, with linearly dependent
//   columns dropped.
//   Rayleigh-Ritz on A = (H - sigma)^2: the projected matrix is the Gram of
//   HS = (H - sigma) S, M = HS^T HS = S^T A S.  Forming it from (H - sigma) S
//   rather than from A S keeps the tiny eigenvalues of the fold accurate to
//   the precision of (H - sigma) S itself.
//   X' = S C (b smallest Ritz pairs), P' = S C^ with C^ the X-free part of C
//   made orthogonal to C and orthonormal in the small space, so
//   [X' P'] is orthonormal without touching the n-length blocks again.
//   Convergence: Rayleigh-Ritz with H itself inside span(X) gives the Ritz
//   values theta of H - sigma; the nev with smallest |theta| are the wanted
//   pairs, accepted when ||(H - sigma) x - theta x||_2 <= tol.  Before
//   returning, the residuals are recomputed with a fresh FP64 apply.
//   Soft locking (option): wanted pairs whose residual is below tol/10 stay
//   in X and in every Rayleigh-Ritz step but get no new W direction, so the
//   inner CG runs on fewer columns once the pairs nearest sigma converge.
//
// Precision (MBL_MIXED): a first phase keeps every n-length block in FP32 (FP32
// applies, FP32 combinations, FP32-MFMA Grams, FP32 PCG) while all small dense
// algebra stays FP64; once that phase reaches 1e-4 or an iteration fails to
// halve the residual, the blocks are promoted to FP64 and the iteration
// continues with FP64 blocks and FP32 PCG until the requested tolerance.
// MBL_PCG32 runs only the second kind of phase, MBL_F64 runs FP64 everywhere.
//
// Spectrum bounds: plain LOBPCG (block 4) on +H and -H with a Davidson-type
// diagonal preconditioner W = R / max(|+-diag(H) - mu|, J/2).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <utility>
#include <vector>

#include "common.h"

namespace mbl {

int chol_drop(int b, const double* G, int64_t ldg, double tol, double* Rinv, double* work,
              int* dcount, hipStream_t s);
void small_gemm(int M, int N, int K, double alpha, const double* A, int64_t lda, bool ta,
                const double* B, int64_t ldb, bool tb, double beta, double* C, int64_t ldc,
                hipStream_t s);
void gather_cols(int rows, int nsel, const int* sel, const double* Z, int64_t ldz, double* out,
                 int64_t ldo, hipStream_t s);

thread_local PhaseClock* t_phase_clock = nullptr;

hipEvent_t PhaseClock::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  MBL_HIP(hipEventCreate(&e));
  return e;
}

void PhaseClock::collect() {
  for (const Pair& p : pend) {
    float t = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&t, p.a, p.b) == hipSuccess)
      ms[p.kind] += t;
    pool.push_back(p.a);
    pool.push_back(p.b);
  }
  pend.clear();
}

PhaseClock::~PhaseClock() {
  for (const Pair& p : pend) {
    (void)hipEventSynchronize(p.b);
    pool.push_back(p.a);
    pool.push_back(p.b);
  }
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

PhaseTick::PhaseTick(int k, hipStream_t st) : c(t_phase_clock), kind(k), s(st) {
  if (!c) return;
  a = c->get();
  if (hipEventRecord(a, s) != hipSuccess) {
    c->pool.push_back(a);
    c = nullptr;
  }
}

PhaseTick::~PhaseTick() {
  if (!c) return;
  hipEvent_t b = nullptr;
  try {
    b = c->get();
  } catch (...) {
    c->pool.push_back(a);
    return;
  }
  if (hipEventRecord(b, s) == hipSuccess) {
    c->pend.push_back({kind, a, b});
  } else {
    c->pool.push_back(a);
    c->pool.push_back(b);
  }
}

namespace {

using clk = std::chrono::steady_clock;
double secs(clk::time_point a) { return std::chrono::duration<double>(clk::now() - a).count(); }

struct Params {
  double sigma = 0;
  int nev = 1, b = 2;
  double tol = 1e-10;
  int max_iter = 400;
  int pcg_iters = 0;
  int verbose = 0;
  uint64_t seed = 0;
  bool fold = true;   // false: plain LOBPCG on sign * (H - sigma)
  double sign = 1.0;
  bool diag_precond = false;  // plain mode: W = R / |sign*diag(H) - mu| instead of W = R
  double lock_tol = 0;        // > 0: soft locking of wanted pairs with residual <= lock_tol
  StopCheck stop;             // deadline / cancel flag of the caller
  bool fold_select = true;    // fold: wanted pairs by their fold quotient (Phase::check)
  double guard_frac = 1.0;    // CG steps of the guard columns, as a fraction of m
};

struct Stats {
  int iters = 0, iters_fp64 = 0;
  bool stopped = false;  // the caller's deadline or cancel flag ended the solve
  int64_t applies = 0, pcg_steps = 0, pcg_columns = 0;
  double t_pcg = 0, t_rr = 0;
  bool timing = false;
  PcgTiming tm[2];  // [0] FP64 inner solves, [1] FP32 inner solves
};

// Small FP64 device workspace of one solve (sizes for m = 3b).
struct Small {
  DevBuf M, V, w, C, Ch, T1, T2, Rinv, cw, ew, sel, cnt, K, Z, th, Zs, asel, Za;
  int mmax;
  Small(int b, hipStream_t s) {
    const int m = 3 * b;
    mmax = m;
    const size_t mm = (size_t)m * m * sizeof(double);
    M.reset(mm, s);
    V.reset(mm, s);
    w.reset(m * sizeof(double), s);
    C.reset(mm, s);
    Ch.reset(mm, s);
    T1.reset(mm, s);
    T2.reset(mm, s);
    Rinv.reset(mm, s);
    cw.reset(mm, s);
    ew.reset(small_eigh_work_bytes(m), s);
    sel.reset(m * sizeof(int), s);
    cnt.reset(64, s);
    K.reset(mm, s);
    Z.reset(mm, s);
    th.reset(m * sizeof(double), s);
    Zs.reset(mm, s);
    asel.reset((size_t)b * sizeof(int), s);
    Za.reset((size_t)b * b * sizeof(double), s);
  }
};

template <class TB>
struct PhaseBufs {
  int64_t n;
  int b, ld;
  DevBuf S[2], HS[2], R, tmp;
  PhaseBufs(int64_t n_, int b_, hipStream_t s) : n(n_), b(b_), ld(3 * b_) {
    for (int i = 0; i < 2; ++i) {
      S[i].reset((size_t)n * ld * sizeof(TB), s);
      HS[i].reset((size_t)n * ld * sizeof(TB), s);
    }
    R.reset((size_t)n * b * sizeof(TB), s);
    tmp.reset((size_t)n * b * sizeof(TB), s);
  }
};

// CG steps per outer iteration.  The total number of CG steps a solve needs is
// nearly independent of this split (measured at L = 20: within 10% for m from
// 125 to 2000); larger m means fewer outer iterations.  40 (n/924)^0.61 gives
// ~1000 at L = 20 and ~5200 at L = 24 (the paper used 5,000 at L = 24).
int default_pcg_iters(int64_t n) {
  const double m = 40.0 * std::pow((double)n / 924.0, 0.61);
  return (int)std::max(5.0, std::min(20000.0, std::round(m)));
}

template <class TB>
double drop_tol() {
  return sizeof(TB) == 8 ? 1e-14 : 1e-6;
}

// Y (n x q, ld ldy) <- cols of a block: copy helper
template <class TB>
void copy_cols(int64_t n, int q, const TB* X, int64_t ldx, TB* Y, int64_t ldy, hipStream_t s) {
  if (n == 0 || q == 0) return;
  MBL_HIP(hipMemcpy2DAsync(Y, ldy * sizeof(TB), X, ldx * sizeof(TB), q * sizeof(TB), n,
                           hipMemcpyDeviceToDevice, s));
}

template <class TB>
class Phase {
 public:
  Phase(const Ham& H, const Params& p, Small& sm, Stats& st, hipStream_t s)
      : H_(H), p_(p), sm_(sm), st_(st), s_(s), B_(H.n, p.b, s) {}

  // Orthonormalise X in place (two Cholesky-QR passes); returns kept width.
  int cholqr2(TB* X, int64_t ldx, int q) {
    for (int pass = 0; pass < 2 && q > 0; ++pass) {
      launch_gram<TB>(H_.n, X, ldx, q, X, ldx, q, sm_.T1.as<double>(), q, s_);
      const int k = chol_drop(q, sm_.T1.as<double>(), q, drop_tol<TB>(), sm_.Rinv.as<double>(),
                              sm_.cw.as<double>(), sm_.cnt.as<int>(), s_);
      // Rinv is q x q with ld q, first k columns meaningful
      launch_combine<TB>(H_.n, X, ldx, q, sm_.Rinv.as<double>(), q, B_.tmp.template as<TB>(), p_.b,
                         k, 0.0, s_);
      copy_cols<TB>(H_.n, k, B_.tmp.template as<TB>(), p_.b, X, ldx, s_);
      q = k;
    }
    return q;
  }

  void apply(const TB* X, int64_t ldx, TB* Y, int64_t ldy, int q) {
    launch_apply<TB>(H_, p_.fold ? p_.sigma : 0.0, X, ldx, Y, ldy, q, s_);
    st_.applies += 1;
  }

  // Start from X0 (n x b).  RR on span(X0).
  void init(const TB* X0, int64_t ldx0) {
    const int b = p_.b;
    TB* S = B_.S[cur_].template as<TB>();
    TB* HS = B_.HS[cur_].template as<TB>();
    copy_cols<TB>(H_.n, b, X0, ldx0, S, B_.ld, s_);
    const int k = cholqr2(S, B_.ld, b);
    if (k < b) fail(MBL_EBREAKDOWN, "starting block is rank deficient");
    apply(S, B_.ld, HS, B_.ld, b);
    bp_ = 0;
    rr(b);
  }

  // Rayleigh-Ritz on span(S[:, 0:mact]); updates X, P (and HX, HP), mu.
  void rr(int mact) {
    const int b = p_.b;
    const int64_t n = H_.n;
    const auto t0 = clk::now();
    TB* S = B_.S[cur_].template as<TB>();
    TB* HS = B_.HS[cur_].template as<TB>();
    TB* S2 = B_.S[1 - cur_].template as<TB>();
    TB* HS2 = B_.HS[1 - cur_].template as<TB>();
    double* M = sm_.M.as<double>();
    if (p_.fold)
      launch_gram<TB>(n, HS, B_.ld, mact, HS, B_.ld, mact, M, mact, s_);
    else
      launch_gram<TB>(n, S, B_.ld, mact, HS, B_.ld, mact, M, mact, s_);
    if (p_.sign != 1.0)
      small_gemm(mact, mact, 0, 0.0, M, mact, false, M, mact, false, p_.sign, M, mact, s_);
    small_eigh(mact, M, mact, sm_.w.as<double>(), sm_.V.as<double>(), mact, sm_.ew.as<double>(),
               s_);
    mu_.resize(b);
    MBL_HIP(hipMemcpyAsync(mu_.data(), sm_.w.as<double>(), b * sizeof(double),
                           hipMemcpyDeviceToHost, s_));
    // C = V[:, 0:b] (mact x b, ld b)
    double* C = sm_.C.as<double>();
    MBL_HIP(hipMemcpy2DAsync(C, b * sizeof(double), sm_.V.as<double>(), mact * sizeof(double),
                             b * sizeof(double), mact, hipMemcpyDeviceToDevice, s_));
    // X' = S C, HX' = HS C
    launch_combine<TB>(n, S, B_.ld, mact, C, b, S2, B_.ld, b, 0.0, s_);
    launch_combine<TB>(n, HS, B_.ld, mact, C, b, HS2, B_.ld, b, 0.0, s_);
    int bp_new = 0;
    if (mact > b) {
      // C^ = C with the X rows zeroed, projected off C twice, orthonormalised.
      double* Ch = sm_.Ch.as<double>();
      MBL_HIP(hipMemcpyAsync(Ch, C, (size_t)mact * b * sizeof(double), hipMemcpyDeviceToDevice,
                             s_));
      MBL_HIP(hipMemsetAsync(Ch, 0, (size_t)b * b * sizeof(double), s_));
      double* T1 = sm_.T1.as<double>();
      for (int pass = 0; pass < 2; ++pass) {
        small_gemm(b, b, mact, 1.0, C, b, true, Ch, b, false, 0.0, T1, b, s_);   // C^T C^
        small_gemm(mact, b, b, -1.0, C, b, false, T1, b, false, 1.0, Ch, b, s_);  // C^ -= C T1
      }
      small_gemm(b, b, mact, 1.0, Ch, b, true, Ch, b, false, 0.0, T1, b, s_);
      const int k = chol_drop(b, T1, b, 1e-14, sm_.Rinv.as<double>(), sm_.cw.as<double>(),
                              sm_.cnt.as<int>(), s_);
      double* T2 = sm_.T2.as<double>();
      small_gemm(mact, k, b, 1.0, Ch, b, false, sm_.Rinv.as<double>(), b, false, 0.0, T2, b, s_);
      launch_combine<TB>(n, S, B_.ld, mact, T2, b, S2 + b, B_.ld, k, 0.0, s_);
      launch_combine<TB>(n, HS, B_.ld, mact, T2, b, HS2 + b, B_.ld, k, 0.0, s_);
      bp_new = k;
    }
    cur_ = 1 - cur_;
    bp_ = bp_new;
    MBL_HIP(hipStreamSynchronize(s_));
    st_.t_rr += secs(t0);
  }

  // H-Rayleigh-Ritz inside span(X): wanted Ritz values (of H - sigma, or of
  // sign*H in plain mode) and residual norms.  Leaves Zsel (b x nev) in sm_.Zs.
  void check(std::vector<double>& theta, std::vector<double>& res) {
    const int b = p_.b, nev = p_.nev;
    const int64_t n = H_.n;
    const auto t0 = clk::now();
    TB* X = B_.S[cur_].template as<TB>();
    TB* HX = B_.HS[cur_].template as<TB>();
    double* K = sm_.K.as<double>();
    launch_gram<TB>(n, X, B_.ld, b, HX, B_.ld, b, K, b, s_);
    if (p_.sign != 1.0) small_gemm(b, b, 0, 0.0, K, b, false, K, b, false, p_.sign, K, b, s_);
    small_eigh(b, K, b, sm_.th.as<double>(), sm_.Z.as<double>(), b, sm_.ew.as<double>(), s_);
    std::vector<double> th_all(b);
    MBL_HIP(hipMemcpyAsync(th_all.data(), sm_.th.as<double>(), b * sizeof(double),
                           hipMemcpyDeviceToHost, s_));
    MBL_HIP(hipStreamSynchronize(s_));
    last_theta_all_ = th_all;
    // residuals of all b H-Ritz pairs: R = sign*HX Z - X Z diag(theta)
    double* Zt = sm_.T1.as<double>();
    MBL_HIP(hipMemcpyAsync(Zt, sm_.Z.as<double>(), (size_t)b * b * sizeof(double),
                           hipMemcpyDeviceToDevice, s_));
    h_Dc_.assign((size_t)b * b, 0.0);
    for (int j = 0; j < b; ++j) h_Dc_[(size_t)j * b + j] = -th_all[j];
    MBL_HIP(hipMemcpyAsync(sm_.T2.get(), h_Dc_.data(), h_Dc_.size() * sizeof(double),
                           hipMemcpyHostToDevice, s_));
    small_gemm(b, b, b, 1.0, sm_.Z.as<double>(), b, false, sm_.T2.as<double>(), b, false, 0.0, Zt, b,
               s_);
    TB* Rr = B_.tmp.template as<TB>();
    if (p_.sign != 1.0) {
      double* Zsg = sm_.Ch.as<double>();
      MBL_HIP(hipMemcpyAsync(Zsg, sm_.Z.as<double>(), (size_t)b * b * sizeof(double),
                             hipMemcpyDeviceToDevice, s_));
      small_gemm(b, b, 0, 0.0, Zsg, b, false, Zsg, b, false, p_.sign, Zsg, b, s_);
      launch_combine<TB>(n, HX, B_.ld, b, Zsg, b, Rr, b, b, 0.0, s_);
    } else {
      launch_combine<TB>(n, HX, B_.ld, b, sm_.Z.as<double>(), b, Rr, b, b, 0.0, s_);
    }
    launch_combine<TB>(n, X, B_.ld, b, Zt, b, Rr, b, b, 1.0, s_);
    launch_gram<TB>(n, Rr, b, b, Rr, b, b, sm_.K.as<double>(), b, s_);
    std::vector<double> G((size_t)b * b);
    MBL_HIP(hipMemcpyAsync(G.data(), sm_.K.as<double>(), G.size() * sizeof(double),
                           hipMemcpyDeviceToHost, s_));
    MBL_HIP(hipStreamSynchronize(s_));
    std::vector<double> r_all(b);
    for (int j = 0; j < b; ++j) r_all[j] = std::sqrt(std::max(0.0, G[(size_t)j * b + j]));
    // The wanted pairs.  Fold: the nev H-Ritz pairs whose vectors x have the
    // smallest fold quotient x^T (H - sigma)^2 x = theta^2 + |r|^2 (r is
    // orthogonal to x).  Selecting by |theta| alone would let an unconverged
    // combination whose H-quotient happens to lie near sigma -- the middle of
    // the spectrum, where such quotients cluster -- take the place of a true
    // eigenvalue at the edge of the window; its fold quotient gives it away.
    // Once the pairs converge (r -> 0) both rules agree.  Plain mode: the nev
    // smallest theta of sign*(H - sigma).
    std::vector<int> sel(nev);
    {
      std::vector<int> ord(b);
      for (int j = 0; j < b; ++j) ord[j] = j;
      if (p_.fold) {
        auto key = [&](int j) {
          return p_.fold_select ? th_all[j] * th_all[j] + r_all[j] * r_all[j] : std::fabs(th_all[j]);
        };
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int c) { return key(a) < key(c); });
        ord.resize(nev);
        std::sort(ord.begin(), ord.end(), [&](int a, int c) { return th_all[a] < th_all[c]; });
      }
      for (int j = 0; j < nev; ++j) sel[j] = ord[j];
    }
    h_sel_ = sel;
    MBL_HIP(hipMemcpyAsync(sm_.sel.get(), h_sel_.data(), nev * sizeof(int), hipMemcpyHostToDevice,
                           s_));
    gather_cols(b, nev, sm_.sel.as<int>(), sm_.Z.as<double>(), b, sm_.Zs.as<double>(), nev, s_);
    theta.resize(nev);
    res.resize(nev);
    for (int j = 0; j < nev; ++j) {
      theta[j] = th_all[sel[j]];
      res[j] = r_all[sel[j]];
    }
    MBL_HIP(hipStreamSynchronize(s_));
    // soft locking: H-Ritz directions (columns of Z) of the wanted pairs
    // below the locking tolerance, most converged first
    locked_.clear();
    if (p_.lock_tol > 0) {
      std::vector<std::pair<double, int>> lk;
      for (int j = 0; j < nev; ++j)
        if (res[j] <= p_.lock_tol) lk.push_back({res[j], sel[j]});
      std::sort(lk.begin(), lk.end());
      for (const auto& e : lk) locked_.push_back(e.second);
    }
    st_.t_rr += secs(t0);
  }

  // Forget the locked set (every direction gets a new W column next step).
  void unlock() { locked_.clear(); }
  int nlocked() const { return (int)locked_.size(); }

  // One LOBPCG step: W from the residual, then RR on [X P W].
  // Returns false when no new direction survived (stagnation).
  template <class TP>
  bool step(const TP* jac, int m) {
    const int b = p_.b;
    const int64_t n = H_.n;
    TB* S = B_.S[cur_].template as<TB>();
    TB* HS = B_.HS[cur_].template as<TB>();
    TB* R = B_.R.template as<TB>();
    TB* W = S + b + bp_;
    const int64_t ld = B_.ld;
    int wq = b;
    const TB* Rin = R;
    int64_t ldRin = b;
    // Columns that get a new direction: all, or with soft locking all but the
    // most converged locked wanted pairs (Z columns), the active width rounded
    // up to whole 128-byte rows of the preconditioner's scalars so the block
    // CG keeps its tuned shapes.
    std::vector<int>& act = h_act_;
    act.clear();
    const int grain = 128 / (int)sizeof(TP);
    int act_wanted = 0;  // unlocked wanted pairs, leading act when guard columns apply
    {
      std::vector<char> drop(b, 0);
      if (p_.fold && m > 0 && !locked_.empty()) {
        int keep = b - (int)locked_.size();
        keep = std::min(b, std::max(grain, (keep + grain - 1) / grain * grain));
        for (int k = 0; k < b - keep; ++k) drop[locked_[k]] = 1;
      }
      if (p_.fold && m > 0 && !locked_.empty() && p_.guard_frac < 1.0) {
        // guard columns with soft locking: the unlocked wanted pairs first (they
        // run every CG step), then the locked ones still active, then the rest
        std::vector<char> wanted(b, 0), locked(b, 0);
        for (int j : h_sel_) wanted[j] = 1;
        for (int j : locked_) locked[j] = 1;
        for (int j = 0; j < b; ++j)
          if (!drop[j] && wanted[j] && !locked[j]) act.push_back(j);
        act_wanted = (int)act.size();
        for (int j = 0; j < b; ++j)
          if (!drop[j] && wanted[j] && locked[j]) act.push_back(j);
        for (int j = 0; j < b; ++j)
          if (!drop[j] && !wanted[j]) act.push_back(j);
      } else {
        for (int j = 0; j < b; ++j)
          if (!drop[j]) act.push_back(j);
      }
    }
    const int keep = (int)act.size();
    const auto t_res = clk::now();
    // A-residual R = sign*(op) applied to HX minus X diag(mu)
    h_D_.assign((size_t)b * b, 0.0);
    for (int j = 0; j < b; ++j) h_D_[(size_t)j * b + j] = -mu_[j];
    MBL_HIP(hipMemcpyAsync(sm_.T2.get(), h_D_.data(), h_D_.size() * sizeof(double),
                           hipMemcpyHostToDevice, s_));
    if (p_.fold) {
      apply(HS, B_.ld, R, b, b);
    } else {
      // R = sign * HX
      h_I_.assign((size_t)b * b, 0.0);
      for (int j = 0; j < b; ++j) h_I_[(size_t)j * b + j] = p_.sign;
      MBL_HIP(hipMemcpyAsync(sm_.T1.get(), h_I_.data(), h_I_.size() * sizeof(double),
                             hipMemcpyHostToDevice, s_));
      launch_combine<TB>(n, HS, B_.ld, b, sm_.T1.as<double>(), b, R, b, b, 0.0, s_);
    }
    launch_combine<TB>(n, S, B_.ld, b, sm_.T2.as<double>(), b, R, b, b, 1.0, s_);
    if (p_.fold && m > 0 && keep < b) {
      TB* Rt = B_.tmp.template as<TB>();
      MBL_HIP(hipMemcpyAsync(sm_.asel.get(), act.data(), keep * sizeof(int),
                             hipMemcpyHostToDevice, s_));
      gather_cols(b, keep, sm_.asel.as<int>(), sm_.Z.as<double>(), b, sm_.Za.as<double>(), keep,
                  s_);
      launch_combine<TB>(n, R, b, b, sm_.Za.as<double>(), keep, Rt, keep, keep, 0.0, s_);
      Rin = Rt;
      ldRin = keep;
      wq = keep;
    }
    MBL_HIP(hipStreamSynchronize(s_));
    st_.t_rr += secs(t_res);
    if (p_.fold && m > 0) {
      const auto t0 = clk::now();
      PcgTiming* tm = st_.timing ? &st_.tm[sizeof(TP) == 4 ? 1 : 0] : nullptr;
      const StopCheck* stop = (p_.stop.has_deadline || p_.stop.flag) ? &p_.stop : nullptr;
      // guard columns (beyond the nev smallest fold Ritz values, which lead R
      // in its A-Ritz order; with soft locking, beyond the unlocked wanted
      // pairs, which lead the rotated block, in whole 128-byte rows) may stop
      // after a fraction of the CG steps
      int m_all = m, keep = -1;
      if (p_.guard_frac < 1.0) {
        const int lead = (Rin == R) ? p_.nev
                                    : std::max(grain, (act_wanted + grain - 1) / grain * grain);
        if (lead < wq && (Rin == R || act_wanted > 0)) {
          m_all = std::max(1, (int)std::lround(p_.guard_frac * m));
          keep = lead;
        }
      }
      if constexpr (std::is_same<TB, TP>::value) {
        run_pcg<TP>(H_, p_.sigma, jac, Rin, ldRin, W, ld, wq, m_all, s_, tm, stop, keep, m);
        MBL_HIP(hipStreamSynchronize(s_));
      } else {
        DevBuf rp((size_t)n * wq * sizeof(TP), s_), wp((size_t)n * wq * sizeof(TP), s_);
        launch_convert<TB, TP>(n, wq, Rin, ldRin, rp.as<TP>(), wq, s_);
        run_pcg<TP>(H_, p_.sigma, jac, rp.as<TP>(), wq, wp.as<TP>(), wq, wq, m_all, s_, tm, stop,
                    keep, m);
        launch_convert<TP, TB>(n, wq, wp.as<TP>(), wq, W, ld, s_);
        MBL_HIP(hipStreamSynchronize(s_));
      }
      st_.applies += 2LL * m;
      st_.pcg_steps += m;
      st_.pcg_columns += keep < 0 ? (int64_t)m * wq
                                  : (int64_t)m_all * wq + (int64_t)(m - m_all) * keep;
      st_.t_pcg += secs(t0);
    } else if constexpr (std::is_same<TB, double>::value) {
      if (!p_.fold && p_.diag_precond) {
        // Davidson-type diagonal preconditioner; the floor J/2 is the size of
        // one flip-flop element, below which the diagonal says nothing
        const double floor = std::max(0.5 * std::fabs(H_.J), 1e-6);
        launch_diag_precond(n, b, R, b, H_.diag.as<double>(), p_.sign, sm_.w.as<double>(), floor,
                            W, ld, s_);
      } else {
        copy_cols<TB>(n, b, R, b, W, ld, s_);
      }
    } else {
      copy_cols<TB>(n, b, R, b, W, ld, s_);
    }
    const auto t0 = clk::now();
    // orthogonalise W against [X P] twice, then Cholesky-QR twice
    const int xp = b + bp_;
    for (int pass = 0; pass < 2; ++pass) {
      launch_gram<TB>(n, S, ld, xp, W, ld, wq, sm_.T1.as<double>(), wq, s_);
      small_gemm(xp, wq, 0, 0.0, sm_.T1.as<double>(), wq, false, sm_.T1.as<double>(), wq, false,
                 -1.0, sm_.T1.as<double>(), wq, s_);  // negate
      launch_combine<TB>(n, S, ld, xp, sm_.T1.as<double>(), wq, W, ld, wq, 1.0, s_);
    }
    const int bw = cholqr2(W, ld, wq);
    st_.t_rr += secs(t0);
    if (bw == 0) return false;
    apply(W, ld, HS + b + bp_, ld, bw);
    rr(b + bp_ + bw);
    return true;
  }

  // Eigen-vectors of the wanted pairs: V = X Zsel (n x nev) in FP64.
  void vectors(double* V, int64_t ldv) {
    const int b = p_.b, nev = p_.nev;
    TB* X = B_.S[cur_].template as<TB>();
    if constexpr (std::is_same<TB, double>::value) {
      launch_combine<double>(H_.n, X, B_.ld, b, sm_.Zs.as<double>(), nev, V, ldv, nev, 0.0, s_);
    } else {
      DevBuf t((size_t)H_.n * nev * sizeof(TB), s_);
      launch_combine<TB>(H_.n, X, B_.ld, b, sm_.Zs.as<double>(), nev, t.as<TB>(), nev, nev, 0.0,
                         s_);
      launch_convert<TB, double>(H_.n, nev, t.as<TB>(), nev, V, ldv, s_);
      MBL_HIP(hipStreamSynchronize(s_));
    }
  }

  // Ritz values of all b columns from the last check() (verbose diagnostics).
  const std::vector<double>& theta_all() const { return last_theta_all_; }

  TB* X() { return B_.S[cur_].template as<TB>(); }
  int64_t ldx() const { return B_.ld; }
  const std::vector<double>& mu() const { return mu_; }

 private:
  const Ham& H_;
  const Params& p_;
  Small& sm_;
  Stats& st_;
  hipStream_t s_;
  PhaseBufs<TB> B_;
  int cur_ = 0;
  int bp_ = 0;
  std::vector<double> mu_;
  std::vector<int> locked_;  // Z columns of locked wanted pairs, most converged first
  std::vector<double> last_theta_all_;
  // host sources of small uploads: members, so that each outlives its
  // asynchronous copy (every upload is followed by a stream synchronisation
  // before the member is written again)
  std::vector<double> h_D_, h_I_, h_Dc_;
  std::vector<int> h_act_, h_sel_;
};

// verbose >= 2: where the wanted pairs stand.  Counts of residuals below
// 1e-4 / 1e-6 / 1e-8 / 1e-10, the ranks (by distance to sigma, 0 = nearest)
// and residuals of the four worst pairs, and the distances to sigma of the
// farthest wanted Ritz value and of the nearest unwanted ones.
void print_detail(const char* tag, int iter, const std::vector<double>& theta,
                  const std::vector<double>& res, const std::vector<double>& th_all) {
  const int nev = (int)theta.size();
  std::vector<int> ord(nev);
  for (int j = 0; j < nev; ++j) ord[j] = j;
  std::sort(ord.begin(), ord.end(),
            [&](int a, int b) { return std::fabs(theta[a]) < std::fabs(theta[b]); });
  std::vector<int> rank(nev);
  for (int r = 0; r < nev; ++r) rank[ord[r]] = r;
  int c4 = 0, c6 = 0, c8 = 0, c10 = 0;
  for (double r : res) {
    c4 += r <= 1e-4;
    c6 += r <= 1e-6;
    c8 += r <= 1e-8;
    c10 += r <= 1e-10;
  }
  std::vector<int> worst(nev);
  for (int j = 0; j < nev; ++j) worst[j] = j;
  std::sort(worst.begin(), worst.end(), [&](int a, int b) { return res[a] > res[b]; });
  std::vector<double> d;
  for (double t : th_all) d.push_back(std::fabs(t));
  std::sort(d.begin(), d.end());
  std::fprintf(stderr, "[mbl %s detail] iter %d below 1e-4/6/8/10: %d %d %d %d; worst (rank:resid)", tag,
               iter, c4, c6, c8, c10);
  for (int k = 0; k < std::min(4, nev); ++k)
    std::fprintf(stderr, " %d:%.2e", rank[worst[k]], res[worst[k]]);
  std::fprintf(stderr, "; |theta| wanted max %.3e, next %.3e %.3e\n", d[nev - 1],
               (int)d.size() > nev ? d[nev] : 0.0, (int)d.size() > nev + 1 ? d[nev + 1] : 0.0);
}

// Fresh FP64 residuals of V (n x nev) with values theta (of H - sigma).
std::vector<double> fresh_residuals(const Ham& H, double sigma, const double* V, int64_t ldv,
                                    int nev, const std::vector<double>& theta, Stats& st,
                                    hipStream_t s) {
  const int64_t n = H.n;
  DevBuf HV((size_t)n * nev * sizeof(double), s), D((size_t)nev * nev * sizeof(double), s),
      G((size_t)nev * nev * sizeof(double), s);
  launch_apply<double>(H, sigma, V, ldv, HV.as<double>(), nev, nev, s);
  st.applies += 1;
  std::vector<double> d((size_t)nev * nev, 0.0);
  for (int j = 0; j < nev; ++j) d[(size_t)j * nev + j] = -theta[j];
  MBL_HIP(hipMemcpyAsync(D.get(), d.data(), d.size() * sizeof(double), hipMemcpyHostToDevice, s));
  launch_combine<double>(n, V, ldv, nev, D.as<double>(), nev, HV.as<double>(), nev, nev, 1.0, s);
  launch_gram<double>(n, HV.as<double>(), nev, nev, HV.as<double>(), nev, nev, G.as<double>(), nev,
                      s);
  std::vector<double> g((size_t)nev * nev);
  MBL_HIP(hipMemcpyAsync(g.data(), G.get(), g.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  MBL_HIP(hipStreamSynchronize(s));
  std::vector<double> r(nev);
  for (int j = 0; j < nev; ++j) r[j] = std::sqrt(std::max(0.0, g[(size_t)j * nev + j]));
  return r;
}

double maxv(const std::vector<double>& v) {
  double m = 0;
  for (double x : v) m = std::max(m, x);
  return m;
}

// Runs LOBPCG iterations of one phase until the wanted residuals are below
// stop_tol, stagnation (if patience > 0: `patience` steps in a row that do not
// bring the largest residual below gain times the best so far) or the
// iteration budget is used.  Returns true on reaching stop_tol.
template <class TB, class TP>
bool run_phase(Phase<TB>& ph, const TP* jac, const Params& p, double stop_tol, int patience,
               double gain, int& iters_left, Stats& st, std::vector<double>& theta,
               std::vector<double>& res, const char* tag) {
  const int m = p.pcg_iters;
  double best = INFINITY;
  int since = 0;
  while (true) {
    ph.check(theta, res);
    if (t_phase_clock) t_phase_clock->collect();  // check() synchronised the stream
    const double r = maxv(res);
    if (p.verbose) {
      if (p.lock_tol > 0)
        std::fprintf(stderr, "[mbl %s] iter %d applies %lld max_resid %.3e locked %d\n", tag,
                     st.iters, (long long)st.applies, r, ph.nlocked());
      else
        std::fprintf(stderr, "[mbl %s] iter %d applies %lld max_resid %.3e\n", tag, st.iters,
                     (long long)st.applies, r);
      if (p.verbose >= 2) print_detail(tag, st.iters, theta, res, ph.theta_all());
    }
    if (r <= stop_tol) return true;
    if (p.stop.triggered()) {
      st.stopped = true;
      return false;
    }
    if (patience > 0) {
      if (r < gain * best) {
        best = r;
        since = 0;
      } else if (++since >= patience) {
        return false;
      }
    }
    if (iters_left <= 0) return false;
    --iters_left;
    ++st.iters;
    if (!ph.step(jac, m)) return false;
  }
}

}  // namespace

// Interior solve.  evals/resid host (nev), evecs device (may be null).
mbl_status solve_interior(const Ham& H, double sigma, int nev, int b, double tol,
                          const mbl_solve_opts& o, double* evals, double* evecs, int64_t ldv,
                          double* resid, mbl_solve_info* info, hipStream_t s) {
  const auto t_start = clk::now();
  Params p;
  p.sigma = sigma;
  p.nev = nev;
  p.b = b;
  p.tol = tol;
  p.max_iter = o.max_iter > 0 ? o.max_iter : 400;
  p.pcg_iters = o.pcg_iters > 0 ? o.pcg_iters : default_pcg_iters(H.n);
  p.verbose = o.verbose;
  p.seed = o.seed;
  p.lock_tol = o.lock ? 0.1 * tol : 0.0;
  // MBL_SELECT=theta: wanted pairs by |theta| alone (for comparison)
  {
    const char* sel = std::getenv("MBL_SELECT");
    p.fold_select = !(sel && sel[0] == 't');
  }
  // guard columns: a fraction of the CG steps where that measured faster (large
  // sectors, and at least 64 wanted columns, so that the CG on them alone
  // still runs on wide rows)
  p.guard_frac = o.guard_cg > 0 ? std::min(1.0, o.guard_cg)
                                : (H.n >= 500000 && nev >= 64 ? 0.05 : 1.0);
  p.stop.flag = o.cancel;
  if (o.max_seconds > 0) {
    p.stop.has_deadline = true;
    p.stop.deadline = t_start + std::chrono::duration_cast<clk::duration>(
                                    std::chrono::duration<double>(o.max_seconds));
  }
  Stats st;
  st.timing = o.timing != 0;
  // phase clock of this solve (this thread) while the solve runs
  PhaseClock clock;
  struct ClockScope {
    PhaseClock* prev;
    explicit ClockScope(PhaseClock* c) : prev(t_phase_clock) { t_phase_clock = c; }
    ~ClockScope() { t_phase_clock = prev; }
  } clock_scope(st.timing ? &clock : nullptr);
  Small sm(b, s);
  const int64_t n = H.n;
  const int prec = o.precision;
  std::vector<double> theta, res;
  int iters_left = p.max_iter;
  DevBuf V((size_t)n * nev * sizeof(double), s);
  DevBuf jac32, jac64;
  bool ok = false;

  DevBuf X0((size_t)n * b * sizeof(double), s);
  launch_randn<double>(n, b, p.seed, X0.as<double>(), b, s);
  if (prec == MBL_MIXED || prec == MBL_PCG32) {
    jac32.reset((size_t)n * sizeof(float), s);
    launch_jacobi<float>(H, sigma, jac32.as<float>(), s);
  }
  if (prec == MBL_F64) {
    jac64.reset((size_t)n * sizeof(double), s);
    launch_jacobi<double>(H, sigma, jac64.as<double>(), s);
  }
  if (prec == MBL_MIXED) {
    // phase 1: FP32 blocks until the FP32 floor
    Phase<float> ph(H, p, sm, st, s);
    {
      DevBuf x32((size_t)n * b * sizeof(float), s);
      launch_convert<double, float>(n, b, X0.as<double>(), b, x32.as<float>(), b, s);
      ph.init(x32.as<float>(), b);
    }
    // The inner CG runs in FP32 in both phases, so an FP32-block iteration
    // costs about as much as an FP64-block one, and the FP64-block phase
    // reduces the residual about twofold per iteration down to the tolerance.
    // Leave the FP32 phase at 1e-4 or at the first iteration that does not
    // halve the residual, whichever comes first.
    const double sw = std::max(tol, 1e-4);
    run_phase<float, float>(ph, jac32.as<float>(), p, sw, 1, 0.5, iters_left, st, theta, res,
                            "fp32");
    launch_convert<float, double>(n, b, ph.X(), ph.ldx(), X0.as<double>(), b, s);
    MBL_HIP(hipStreamSynchronize(s));
  }
  {
    Phase<double> ph(H, p, sm, st, s);
    ph.init(X0.as<double>(), b);
    X0.release();
    const int it0 = st.iters;
    while (true) {
      bool reached;
      if (prec == MBL_F64)
        reached = run_phase<double, double>(ph, jac64.as<double>(), p, tol, 0, 0.0, iters_left, st,
                                            theta, res, "fp64");
      else
        reached = run_phase<double, float>(ph, jac32.as<float>(), p, tol, 0, 0.0, iters_left, st, theta,
                                           res, "fp64/pcg32");
      ph.vectors(V.as<double>(), nev);
      res = fresh_residuals(H, sigma, V.as<double>(), nev, nev, theta, st, s);
      ok = reached && maxv(res) <= tol;
      if (ok || !reached || iters_left <= 0 || st.stopped) break;
      // tracked residuals passed but fresh ones did not: one more step, with
      // every direction active
      ph.unlock();
      --iters_left;
      ++st.iters;
      bool stepped;
      if (prec == MBL_F64)
        stepped = ph.step(jac64.as<double>(), p.pcg_iters);
      else
        stepped = ph.step(jac32.as<float>(), p.pcg_iters);
      if (!stepped) break;
    }
    st.iters_fp64 = (prec == MBL_MIXED) ? st.iters - it0 : st.iters;
  }
  // outputs, ascending theta already
  for (int j = 0; j < nev; ++j) {
    evals[j] = theta[j] + sigma;
    if (resid) resid[j] = res[j];
  }
  if (evecs)
    MBL_HIP(hipMemcpy2DAsync(evecs, ldv * sizeof(double), V.get(), nev * sizeof(double),
                             nev * sizeof(double), n, hipMemcpyDeviceToDevice, s));
  MBL_HIP(hipStreamSynchronize(s));
  if (st.timing) clock.collect();
  if (info) {
    info->iters = st.iters;
    info->iters_fp64 = st.iters_fp64;
    info->applies = st.applies;
    info->pcg_steps = st.pcg_steps;
    info->pcg_columns = st.pcg_columns;
    info->t_pcg = st.t_pcg;
    info->t_rr = st.t_rr;
    info->max_resid = maxv(res);
    int nc = 0;
    for (double r : res) nc += (r <= tol);
    info->nconv = nc;
    info->seconds = secs(t_start);
    for (int k = 0; k < 2; ++k) {
      info->cg_apply1_launches[k] = st.tm[k].launches[0];
      info->cg_apply2_launches[k] = st.tm[k].launches[1];
      info->cg_apply1_ms[k] = st.tm[k].ms[0];
      info->cg_apply2_ms[k] = st.tm[k].ms[1];
      info->cg_apply1_bytes[k] = st.tm[k].bytes[0];
      info->cg_apply2_bytes[k] = st.tm[k].bytes[1];
      if (st.tm[k].split) info->cg_split = 1;
      info->cg_launches_all[k] = st.tm[k].launches_all;
      info->cg_apply1_ms_all[k] = st.tm[k].ms_all[0];
      info->cg_apply2_ms_all[k] = st.tm[k].ms_all[1];
      info->cg_apply1_bytes_all[k] = st.tm[k].bytes_all[0];
      info->cg_apply2_bytes_all[k] = st.tm[k].bytes_all[1];
    }
    info->t_apply = 1e-3 * clock.ms[PhaseClock::APPLY];
    info->t_gram = 1e-3 * clock.ms[PhaseClock::GRAM];
    info->t_small = 1e-3 * clock.ms[PhaseClock::SMALL];
  }
  if (ok) return MBL_OK;
  return st.stopped ? MBL_ECANCELLED : MBL_ENOCONV;
}

// Extreme eigenvalues by plain LOBPCG on +H and -H (block 4, no preconditioner).
mbl_status spectrum_bounds(const Ham& H, double tol, double* emin, double* emax, hipStream_t s) {
  const int64_t n = H.n;
  const int b = (int)std::min<int64_t>(4, n / 2 > 0 ? n / 2 : 1);
  if (n <= 2) {
    // tiny sectors: Rayleigh-Ritz on the identity basis is exact
    Params p;
    p.fold = false;
    p.b = (int)n;
    p.nev = (int)n;
    Stats st;
    Small sm((int)n, s);
    DevBuf I((size_t)n * n * sizeof(double), s);
    std::vector<double> e((size_t)n * n, 0.0);
    for (int64_t i = 0; i < n; ++i) e[(size_t)i * n + i] = 1.0;
    MBL_HIP(hipMemcpyAsync(I.get(), e.data(), e.size() * sizeof(double), hipMemcpyHostToDevice, s));
    DevBuf HI((size_t)n * n * sizeof(double), s);
    launch_apply<double>(H, 0.0, I.as<double>(), n, HI.as<double>(), n, (int)n, s);
    std::vector<double> hm((size_t)n * n);
    MBL_HIP(hipMemcpyAsync(hm.data(), HI.get(), hm.size() * sizeof(double), hipMemcpyDeviceToHost,
                           s));
    MBL_HIP(hipStreamSynchronize(s));
    if (n == 1) {
      *emin = *emax = hm[0];
    } else {
      const double a = hm[0], d = hm[3], c = hm[1];
      const double mid = 0.5 * (a + d), rad = std::sqrt(0.25 * (a - d) * (a - d) + c * c);
      *emin = mid - rad;
      *emax = mid + rad;
    }
    return MBL_OK;
  }
  double out[2];
  for (int k = 0; k < 2; ++k) {
    Params p;
    p.fold = false;
    p.sign = k == 0 ? 1.0 : -1.0;
    p.diag_precond = true;
    p.b = b;
    p.nev = 1;
    p.seed = 12345 + k;
    Stats st;
    Small sm(b, s);
    Phase<double> ph(H, p, sm, st, s);
    DevBuf X0((size_t)n * b * sizeof(double), s);
    launch_randn<double>(n, b, p.seed, X0.as<double>(), b, s);
    ph.init(X0.as<double>(), b);
    std::vector<double> theta, res;
    int left = 5000;
    // residual r bounds the eigenvalue error by r^2 / gap for an extreme pair
    const double rtol = std::max(1e-9, std::sqrt(tol) * 1e-2);
    run_phase<double, double>(ph, (const double*)nullptr, p, rtol, 0, 0.0, left, st, theta, res,
                              "bounds");
    out[k] = p.sign * theta[0];
  }
  *emin = out[0];
  *emax = out[1];
  return MBL_OK;
}

}  // namespace mbl
