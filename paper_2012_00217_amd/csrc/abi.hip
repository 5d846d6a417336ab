// extern "C" boundary of libmbl: argument validation, status codes,
// thread-local error messages and the allocator hook.  Every entry point
// catches everything: no exception crosses the C ABI.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "common.h"

namespace mbl {
namespace {

thread_local std::string g_last_error;
mbl_alloc_fn g_alloc = nullptr;
mbl_free_fn g_free = nullptr;
void* g_ctx = nullptr;

template <class F>
mbl_status guard(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.status;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return MBL_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return MBL_EINTERNAL;
  } catch (...) {
    g_last_error = "unknown failure";
    return MBL_EINTERNAL;
  }
}

void require(bool ok, const char* what) {
  if (!ok) fail(MBL_EINVAL, what);
}

const Ham& ham(mbl_ham h) {
  require(h != nullptr, "null Hamiltonian handle");
  return *reinterpret_cast<const Ham*>(h);
}

bool block_prec(int p) { return p == MBL_F64 || p == MBL_F32; }

}  // namespace

namespace {
std::mutex g_pool_mu;
bool g_pool_ready[64] = {};

// Keep freed stream-ordered memory in the device pool instead of returning it
// to the driver at every synchronisation (once per device).
void prepare_pool() {
  int dev = 0;
  MBL_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (g_pool_ready[dev]) return;
  hipMemPool_t pool;
  MBL_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
  uint64_t keep = UINT64_MAX;
  MBL_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
  g_pool_ready[dev] = true;
}
}  // namespace

void* dev_alloc(size_t bytes, hipStream_t s, bool ordered, AllocOwner* owner) {
  void* p = nullptr;
  owner->s = s;
  owner->ordered = ordered;
  if (g_alloc) {
    p = g_alloc(bytes, s, g_ctx);
    if (!p) fail(MBL_ENOMEM, "allocator callback returned NULL for " + std::to_string(bytes) + " bytes");
    owner->free_fn = g_free;
    owner->ctx = g_ctx;
    return p;
  }
  owner->free_fn = nullptr;
  owner->ctx = nullptr;
  if (ordered) {
    prepare_pool();
    MBL_HIP(hipMallocAsync(&p, bytes, s));
  } else {
    MBL_HIP(hipMalloc(&p, bytes));
  }
  return p;
}

void dev_free(void* p, const AllocOwner& o) {
  if (!p) return;
  if (o.free_fn) {
    o.free_fn(p, o.s, o.ctx);
    return;
  }
  if (o.ordered)
    (void)hipFreeAsync(p, o.s);
  else
    (void)hipFree(p);
}

Ham* create_ham(int L, double Sz, double J, double Delta, const double* h_host, hipStream_t stream,
                hipStream_t home) {
  require(L >= 2 && L <= kMaxL, "L must be in [2, 32]");
  require(std::isfinite(Sz) && std::isfinite(J) && std::isfinite(Delta), "Sz, J, Delta must be finite");
  const double two = 2.0 * Sz;
  require(two == std::round(two), "2*Sz must be an integer");
  const long long tsz = (long long)std::llround(two);
  require(((tsz + L) % 2 + 2) % 2 == 0, "2*Sz must have the parity of L");
  require(std::fabs(Sz) <= 0.5 * L, "|Sz| must be <= L/2");
  require(h_host != nullptr, "h is NULL");
  for (int i = 0; i < L; ++i) require(std::isfinite(h_host[i]), "h must be finite");
  auto* H = new Ham();
  H->home = home;
  try {
    H->L = L;
    H->nup = (int)((tsz + L) / 2);
    H->J = J;
    H->Delta = Delta;
    H->hsum = 0;
    for (int i = 0; i < L; ++i) {
      H->h[i] = h_host[i];
      H->hsum += h_host[i];
    }
    const auto C = pascal_table();
    H->n = C[L * kPascal + H->nup];
    build_tables(*H, stream);
    MBL_HIP(hipStreamSynchronize(stream));
  } catch (...) {
    delete H;
    throw;
  }
  return H;
}

int64_t sector_dim(int L, double Sz) {
  require(L >= 2 && L <= kMaxL, "L must be in [2, 32]");
  const double two = 2.0 * Sz;
  require(std::isfinite(Sz) && two == std::round(two), "2*Sz must be an integer");
  const long long tsz = (long long)std::llround(two);
  require(((tsz + L) % 2 + 2) % 2 == 0 && std::fabs(Sz) <= 0.5 * L, "no such sector");
  const auto C = pascal_table();
  return C[L * kPascal + (int)((tsz + L) / 2)];
}

}  // namespace mbl

using namespace mbl;

extern "C" {

const char* mbl_last_error(void) { return g_last_error.c_str(); }

int mbl_version(void) { return 10000; }

mbl_status mbl_set_allocator(mbl_alloc_fn alloc, mbl_free_fn free_fn, void* ctx) {
  return guard([&] {
    require((alloc == nullptr) == (free_fn == nullptr), "allocator: give both callbacks or neither");
    g_alloc = alloc;
    g_free = free_fn;
    g_ctx = ctx;
    return MBL_OK;
  });
}

mbl_status mbl_hamiltonian_create(int L, double Sz, double J, double Delta, const double* h_host,
                                  hipStream_t stream, mbl_ham* out) {
  return guard([&] {
    require(out != nullptr, "out is NULL");
    *out = nullptr;
    Ham* H = create_ham(L, Sz, J, Delta, h_host, stream);
    *out = reinterpret_cast<mbl_ham>(H);
    return MBL_OK;
  });
}

mbl_status mbl_hamiltonian_destroy(mbl_ham h) {
  return guard([&] {
    // kernels of any stream may still read the tables
    if (h) MBL_HIP(hipDeviceSynchronize());
    delete reinterpret_cast<Ham*>(h);
    return MBL_OK;
  });
}

mbl_status mbl_hamiltonian_dim(mbl_ham h, int64_t* n) {
  return guard([&] {
    require(n != nullptr, "n is NULL");
    *n = ham(h).n;
    return MBL_OK;
  });
}

// A non-blocking stream for the entry points that take none: work on the
// legacy stream would have to wait for (or break) hipGraph captures that other
// threads of the process may have in progress.
struct PrivateStream {
  hipStream_t s = nullptr;
  PrivateStream() { MBL_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking)); }
  ~PrivateStream() {
    if (s) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  }
};

mbl_status mbl_sector_states(mbl_ham h, uint64_t* states_host) {
  return guard([&] {
    const Ham& H = ham(h);
    require(states_host != nullptr, "states is NULL");
    std::vector<uint32_t> tmp((size_t)H.n);
    PrivateStream ps;
    MBL_HIP(hipMemcpyAsync(tmp.data(), H.states.get(), (size_t)H.n * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, ps.s));
    MBL_HIP(hipStreamSynchronize(ps.s));
    for (int64_t i = 0; i < H.n; ++i) states_host[i] = tmp[(size_t)i];
    return MBL_OK;
  });
}

mbl_status mbl_rank(mbl_ham h, const uint64_t* states_host, int64_t count, int64_t* idx_host) {
  return guard([&] {
    const Ham& H = ham(h);
    require(count >= 0, "count < 0");
    if (count == 0) return MBL_OK;
    require(states_host && idx_host, "NULL array");
    PrivateStream ps;
    {
      DevBuf q((size_t)count * sizeof(uint64_t), ps.s), r((size_t)count * sizeof(int64_t), ps.s);
      MBL_HIP(hipMemcpyAsync(q.get(), states_host, q.bytes(), hipMemcpyHostToDevice, ps.s));
      rank_states(H, q.as<uint64_t>(), count, r.as<int64_t>(), ps.s);
      MBL_HIP(hipMemcpyAsync(idx_host, r.get(), r.bytes(), hipMemcpyDeviceToHost, ps.s));
      MBL_HIP(hipStreamSynchronize(ps.s));
    }
    return MBL_OK;
  });
}

mbl_status mbl_diagonal(mbl_ham h, double sigma, double* diag_dev, double* jacobi_dev, hipStream_t s) {
  return guard([&] {
    const Ham& H = ham(h);
    require(std::isfinite(sigma), "sigma must be finite");
    if (diag_dev)
      MBL_HIP(hipMemcpyAsync(diag_dev, H.diag.get(), (size_t)H.n * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (jacobi_dev) launch_jacobi<double>(H, sigma, jacobi_dev, s);
    return MBL_OK;
  });
}

static void check_block(const void* X, int64_t ld, int b, const char* name) {
  require(X != nullptr, name);
  require(ld >= b, "leading dimension < b");
}

mbl_status mbl_apply_block(mbl_ham h, double sigma, mbl_precision prec, const void* X, int64_t ldx,
                           void* Y, int64_t ldy, int b, hipStream_t s) {
  return guard([&] {
    const Ham& H = ham(h);
    require(std::isfinite(sigma), "sigma must be finite");
    require(block_prec(prec), "precision must be MBL_F64 or MBL_F32");
    require(b >= 1, "b < 1");
    check_block(X, ldx, b, "X is NULL");
    check_block(Y, ldy, b, "Y is NULL");
    require(X != Y, "X and Y must not overlap");
    if (prec == MBL_F64)
      launch_apply<double>(H, sigma, static_cast<const double*>(X), ldx, static_cast<double*>(Y), ldy, b, s);
    else
      launch_apply<float>(H, sigma, static_cast<const float*>(X), ldx, static_cast<float*>(Y), ldy, b, s);
    return MBL_OK;
  });
}

mbl_status mbl_fold_apply(mbl_ham h, double sigma, mbl_precision prec, const void* X, int64_t ldx,
                          void* T, int64_t ldt, void* Y, int64_t ldy, int b, hipStream_t s) {
  return guard([&] {
    const Ham& H = ham(h);
    require(std::isfinite(sigma), "sigma must be finite");
    require(block_prec(prec), "precision must be MBL_F64 or MBL_F32");
    require(b >= 1, "b < 1");
    check_block(X, ldx, b, "X is NULL");
    check_block(T, ldt, b, "T is NULL");
    check_block(Y, ldy, b, "Y is NULL");
    require(X != T && T != Y, "buffers must not overlap");
    if (prec == MBL_F64) {
      launch_apply<double>(H, sigma, static_cast<const double*>(X), ldx, static_cast<double*>(T), ldt, b, s);
      launch_apply<double>(H, sigma, static_cast<const double*>(T), ldt, static_cast<double*>(Y), ldy, b, s);
    } else {
      launch_apply<float>(H, sigma, static_cast<const float*>(X), ldx, static_cast<float*>(T), ldt, b, s);
      launch_apply<float>(H, sigma, static_cast<const float*>(T), ldt, static_cast<float*>(Y), ldy, b, s);
    }
    return MBL_OK;
  });
}

mbl_status mbl_pcg(mbl_ham h, double sigma, mbl_precision prec, const void* R, int64_t ldr, void* W,
                   int64_t ldw, int b, int m, hipStream_t s) {
  return guard([&] {
    const Ham& H = ham(h);
    require(std::isfinite(sigma), "sigma must be finite");
    require(block_prec(prec), "precision must be MBL_F64 or MBL_F32");
    require(b >= 1 && m >= 0, "b < 1 or m < 0");
    check_block(R, ldr, b, "R is NULL");
    check_block(W, ldw, b, "W is NULL");
    require(R != W, "R and W must not overlap");
    if (prec == MBL_F64) {
      DevBuf jac((size_t)H.n * sizeof(double), s);
      launch_jacobi<double>(H, sigma, jac.as<double>(), s);
      run_pcg<double>(H, sigma, jac.as<double>(), static_cast<const double*>(R), ldr, static_cast<double*>(W), ldw, b, m, s);
    } else {
      DevBuf jac((size_t)H.n * sizeof(float), s);
      launch_jacobi<float>(H, sigma, jac.as<float>(), s);
      run_pcg<float>(H, sigma, jac.as<float>(), static_cast<const float*>(R), ldr, static_cast<float*>(W), ldw, b, m, s);
    }
    MBL_HIP(hipStreamSynchronize(s));
    return MBL_OK;
  });
}

mbl_status mbl_gram(mbl_precision prec, int64_t n, const void* A, int64_t lda, int p, const void* B,
                    int64_t ldb, int q, double* C_dev, int64_t ldc, hipStream_t s) {
  return guard([&] {
    require(block_prec(prec), "precision must be MBL_F64 or MBL_F32");
    require(n >= 0 && p >= 1 && q >= 1, "bad sizes");
    check_block(A, lda, p, "A is NULL");
    check_block(B, ldb, q, "B is NULL");
    require(C_dev != nullptr && ldc >= q, "bad C");
    if (prec == MBL_F64)
      launch_gram<double>(n, static_cast<const double*>(A), lda, p, static_cast<const double*>(B), ldb, q, C_dev, ldc, s);
    else
      launch_gram<float>(n, static_cast<const float*>(A), lda, p, static_cast<const float*>(B), ldb, q, C_dev, ldc, s);
    return MBL_OK;
  });
}

mbl_status mbl_gram_noalloc(mbl_precision prec, int64_t n, const void* A, int64_t lda, int p,
                            const void* B, int64_t ldb, int q, double* C_dev, int64_t ldc,
                            hipStream_t s) {
  return guard([&] {
    require(block_prec(prec), "precision must be MBL_F64 or MBL_F32");
    require(n >= 0 && p >= 1 && q >= 1, "bad sizes");
    check_block(A, lda, p, "A is NULL");
    check_block(B, ldb, q, "B is NULL");
    require(C_dev != nullptr && ldc >= q, "bad C");
    const GramPlan g = gram_plan(n, p, q, A == B && lda == ldb);
    if (g.part_bytes > kGramScratchBytes)
      fail(MBL_EINVAL, "mbl_gram_noalloc: this shape needs " + std::to_string(g.part_bytes) +
                           " bytes of partial sums, above the fixed " +
                           std::to_string(kGramScratchBytes) + " (use mbl_gram)");
    double* part = gram_scratch();
    if (prec == MBL_F64)
      launch_gram_part<double>(g, n, static_cast<const double*>(A), lda, p,
                               static_cast<const double*>(B), ldb, q, C_dev, ldc, part, s);
    else
      launch_gram_part<float>(g, n, static_cast<const float*>(A), lda, p,
                              static_cast<const float*>(B), ldb, q, C_dev, ldc, part, s);
    return MBL_OK;
  });
}

mbl_status mbl_block_combine(mbl_precision prec, int64_t n, const void* A, int64_t lda, int p,
                             const double* C_dev, int64_t ldc, void* Y, int64_t ldy, int q, hipStream_t s) {
  return guard([&] {
    require(block_prec(prec), "precision must be MBL_F64 or MBL_F32");
    require(n >= 0 && p >= 1 && q >= 1, "bad sizes");
    check_block(A, lda, p, "A is NULL");
    check_block(Y, ldy, q, "Y is NULL");
    require(C_dev != nullptr && ldc >= q, "bad C");
    require(A != Y, "A and Y must not overlap");
    if (prec == MBL_F64)
      launch_combine<double>(n, static_cast<const double*>(A), lda, p, C_dev, ldc, static_cast<double*>(Y), ldy, q, 0.0, s);
    else
      launch_combine<float>(n, static_cast<const float*>(A), lda, p, C_dev, ldc, static_cast<float*>(Y), ldy, q, 0.0, s);
    return MBL_OK;
  });
}

mbl_status mbl_small_eigh(int m, const double* A_dev, int64_t lda, double* w_dev, double* V_dev,
                          int64_t ldv, hipStream_t s) {
  return guard([&] {
    require(m >= 1 && m <= 1024, "m must be in [1, 1024]");
    require(A_dev && w_dev && V_dev, "NULL argument");
    require(lda >= m && ldv >= m, "leading dimension < m");
    DevBuf work(small_eigh_work_bytes(m), s);
    small_eigh(m, A_dev, lda, w_dev, V_dev, ldv, work.as<double>(), s);
    MBL_HIP(hipStreamSynchronize(s));
    return MBL_OK;
  });
}

mbl_status mbl_spectrum_bounds(mbl_ham h, double tol, double* emin, double* emax, hipStream_t s) {
  return guard([&] {
    const Ham& H = ham(h);
    require(emin && emax, "NULL output");
    require(tol >= 1e-14 && std::isfinite(tol), "tol must be >= 1e-14");
    return spectrum_bounds(H, tol, emin, emax, s);
  });
}

mbl_status mbl_solve_opts_default(mbl_solve_opts* o) {
  return guard([&] {
    require(o != nullptr, "NULL opts");
    std::memset(o, 0, sizeof(*o));
    o->max_iter = 400;
    o->pcg_iters = 0;
    o->precision = MBL_F64;
    o->verbose = 0;
    o->seed = 0x5eed;
    return MBL_OK;
  });
}

mbl_status mbl_lobpcg_solve(mbl_ham h, double sigma, int nev, int block, double tol,
                            const mbl_solve_opts* opts, double* evals_host, double* evecs_dev,
                            int64_t ldv, double* resid_host, mbl_solve_info* info, hipStream_t s) {
  return guard([&] {
    const Ham& H = ham(h);
    require(std::isfinite(sigma), "sigma must be finite");
    require(nev >= 1 && nev <= block, "need 1 <= nev <= block");
    require(2 * (int64_t)block <= H.n, "need 2 * block <= n");
    require(block <= 320, "block must be <= 320");
    require(tol > 0 && std::isfinite(tol), "tol must be > 0");
    require(evals_host != nullptr, "evals is NULL");
    require(evecs_dev == nullptr || ldv >= nev, "ldv < nev");
    mbl_solve_opts o;
    mbl_solve_opts_default(&o);
    if (opts) o = *opts;
    require(o.precision == MBL_F64 || o.precision == MBL_MIXED || o.precision == MBL_PCG32,
            "precision must be MBL_F64, MBL_MIXED or MBL_PCG32");
    require(o.max_iter >= 0 && o.pcg_iters >= 0, "negative iteration count");
    require(std::isfinite(o.max_seconds) && o.max_seconds >= 0, "max_seconds must be >= 0");
    require(std::isfinite(o.guard_cg) && o.guard_cg >= 0 && o.guard_cg <= 1,
            "guard_cg must be in [0, 1]");
    if (info) std::memset(info, 0, sizeof(*info));
    return solve_interior(H, sigma, nev, block, tol, o, evals_host, evecs_dev, ldv, resid_host, info, s);
  });
}

mbl_status mbl_entanglement_entropy(mbl_ham h, const double* V_dev, int64_t ldv, int nev,
                                    int cut, double* S_host, hipStream_t s) {
  return guard([&] {
    const Ham& H = ham(h);
    require(V_dev && S_host, "NULL argument");
    require(nev >= 1 && ldv >= nev, "need nev >= 1 and ldv >= nev");
    require(cut >= 1 && cut <= H.L - 1 && H.L - cut <= 26, "need 1 <= cut <= L-1, L-cut <= 26");
    entanglement_entropy(H, V_dev, ldv, nev, cut, S_host, s);
    return MBL_OK;
  });
}

mbl_status mbl_gap_ratio(const double* evals_host, int count, double* mean_r) {
  return guard([&] {
    require(evals_host && mean_r, "NULL argument");
    require(count >= 3, "count < 3");
    for (int i = 0; i < count; ++i) require(std::isfinite(evals_host[i]), "non-finite eigenvalue");
    *mean_r = mean_gap_ratio(evals_host, count);
    return MBL_OK;
  });
}

mbl_status mbl_slices_solve(mbl_ham h, int count, const double* sigmas_host, int nev, int block,
                            double tol, const mbl_solve_opts* opts, double* evals_host,
                            double* resid_host, int concurrency) {
  return guard([&] {
    const Ham& H = ham(h);
    require(count >= 1 && sigmas_host && evals_host, "bad arguments");
    for (int i = 0; i < count; ++i) require(std::isfinite(sigmas_host[i]), "sigma must be finite");
    require(nev >= 1 && nev <= block && 2 * (int64_t)block <= H.n && block <= 320, "bad nev/block");
    require(tol > 0 && std::isfinite(tol), "tol must be > 0");
    require(concurrency >= 1, "concurrency < 1");
    mbl_solve_opts o;
    mbl_solve_opts_default(&o);
    if (opts) o = *opts;
    require(o.precision == MBL_F64 || o.precision == MBL_MIXED || o.precision == MBL_PCG32,
            "bad precision");
    return solve_slices(H, count, sigmas_host, nev, block, tol, o, evals_host, resid_host,
                        concurrency);
  });
}

mbl_status mbl_footprint_bytes(int L, double Sz, int block, int precision, size_t* bytes) {
  return guard([&] {
    require(bytes != nullptr, "bytes is NULL");
    require(block >= 1, "block < 1");
    require(precision == MBL_F64 || precision == MBL_MIXED || precision == MBL_PCG32, "bad precision");
    *bytes = solve_footprint(L, Sz, block, precision);
    return MBL_OK;
  });
}

mbl_status mbl_batch_solve(int count, const mbl_problem* problems, mbl_result* results,
                           int concurrency) {
  return guard([&] {
    require(count >= 0, "count < 0");
    if (count == 0) return MBL_OK;
    require(problems != nullptr && results != nullptr, "NULL arrays");
    require(concurrency >= 1, "concurrency < 1");
    return batch_solve(count, problems, results, concurrency);
  });
}

struct mbl_server_s {};

mbl_status mbl_server_create(int device, size_t hbm_budget, int max_slots, mbl_server* out) {
  return guard([&] {
    require(out != nullptr, "out is NULL");
    require(max_slots >= 1 && max_slots <= 64, "max_slots must be in [1, 64]");
    int ndev = 0;
    MBL_HIP(hipGetDeviceCount(&ndev));
    require(device >= 0 && device < ndev, "no such device");
    Server* srv = nullptr;
    server_create(device, max_slots, hbm_budget, &srv);
    *out = reinterpret_cast<mbl_server>(srv);
    return MBL_OK;
  });
}

mbl_status mbl_server_submit(mbl_server srv, const mbl_problem* request, uint64_t* ticket) {
  return guard([&] {
    require(srv && request && ticket, "NULL argument");
    return server_submit(reinterpret_cast<Server*>(srv), request, ticket);
  });
}

mbl_status mbl_server_wait(mbl_server srv, uint64_t ticket, double timeout_s, mbl_result* out) {
  return guard([&] {
    require(srv && out, "NULL argument");
    return server_wait(reinterpret_cast<Server*>(srv), ticket, timeout_s, out);
  });
}

mbl_status mbl_server_cancel(mbl_server srv, uint64_t ticket) {
  return guard([&] {
    require(srv != nullptr, "NULL server");
    return server_cancel(reinterpret_cast<Server*>(srv), ticket);
  });
}

mbl_status mbl_server_stats_get(mbl_server srv, mbl_server_stats* st) {
  return guard([&] {
    require(srv && st, "NULL argument");
    return server_stats(reinterpret_cast<Server*>(srv), st);
  });
}

mbl_status mbl_server_destroy(mbl_server srv) {
  return guard([&] {
    if (srv) server_destroy(reinterpret_cast<Server*>(srv));
    return MBL_OK;
  });
}

}  // extern "C"
