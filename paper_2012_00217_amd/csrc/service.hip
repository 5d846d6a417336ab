// Many independent interior solves on one GPU: a batch call and a serving
// loop with continuous batching (paper Sec. 3.1: disorder realisations,
// disorder strengths and spectral regions are independent, so one GPU can
// run several solves side by side).
//
// Each solve runs on a worker thread with its own non-blocking stream; the
// library's work buffers are stream-ordered, so concurrent solves never wait
// on each other.  A solve is the same deterministic kernel sequence whether it
// runs alone or beside others (fixed-order reductions, no atomics in the
// numerics), so results do not depend on the mix.
//
// Admission (server): requests are taken in arrival order; the head request
// starts as soon as a worker is idle and the sum of the footprints of running
// requests plus its own stays within the budget.  The footprint model counts
// the n-length blocks a solve holds at its peak.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include <tuple>

#include "common.h"

namespace mbl {
namespace {

using clk = std::chrono::steady_clock;

size_t footprint(int64_t n, int b, int prec) {
  // LOBPCG: S and HS double-buffered (4 x 3b columns), residual and scratch
  // (2b), starting block and eigenvectors (2b, FP64); PCG: r, p, T (3b) plus
  // the converted right-hand side and solution (2b) when the PCG runs in a
  // narrower type; per row: state (4 B), diagonal (8 B), Jacobi (8 B).
  auto phase = [&](int sb, int sp) {
    double cols = 14.0 * b * sb + 3.0 * b * sp + (sb != sp ? 2.0 * b * sp : 0.0);
    return cols + 16.0 * b + 20.0;
  };
  double per_row = 0;
  if (prec == MBL_F64) per_row = phase(8, 8);
  else if (prec == MBL_PCG32) per_row = phase(8, 4);
  else per_row = std::max(phase(4, 4), phase(8, 4));
  const double small = 12.0 * (9.0 * b * b * 8.0) + (64 << 20);
  return (size_t)(per_row * (double)n + small);
}

struct Job {
  mbl_problem p{};
  std::vector<double> h;
  uint64_t ticket = 0;
  clk::time_point submitted;
  size_t fp = 0;
  // results
  bool done = false;
  mbl_result r{};
  std::vector<double> evals, resid;
  DevBuf V;  // server: eigenvectors kept until wait()
  int64_t n = 0;
  volatile int cancel = 0;  // set by mbl_server_cancel while the solve runs
};

// One complete solve of a problem on stream s.  Writes evals/resid into the
// job's vectors, vectors into `evecs` (device, may be null).  `cancellable`:
// the solve watches the job's cancel flag (server requests; batch problems
// cannot be cancelled, and their CG steps then run without stop checks).
void run_problem(Job& j, double* evecs, int64_t ldv, hipStream_t s, bool cancellable) {
  const auto t0 = clk::now();
  mbl_result& r = j.r;
  try {
    const mbl_problem& p = j.p;
    // tables stream-ordered on the worker's stream: freeing them never waits
    // for the other workers' work
    std::unique_ptr<Ham> H(create_ham(p.L, p.Sz, p.J, p.Delta, j.h.data(), s, s));
    j.n = H->n;
    if (p.nev < 1 || p.nev > p.block || 2 * (int64_t)p.block > H->n || p.block > 320 ||
        !(p.tol > 0) || !std::isfinite(p.tol))
      fail(MBL_EINVAL, "bad nev/block/tol for this sector");
    double sigma = p.sigma;
    if (p.eps >= 0) {
      double lo = 0, hi = 0;
      spectrum_bounds(*H, 1e-12, &lo, &hi, s);
      sigma = lo + p.eps * (hi - lo);
    }
    if (!std::isfinite(sigma)) fail(MBL_EINVAL, "sigma must be finite");
    mbl_solve_opts o{};
    o.max_iter = p.max_iter > 0 ? p.max_iter : 400;
    o.pcg_iters = p.pcg_iters;
    o.precision = p.precision;
    o.seed = p.seed ? p.seed : 0x5eed;
    // MBL_VERBOSE=1: one stderr line per outer iteration of every solve
    const char* verbose = std::getenv("MBL_VERBOSE");
    o.verbose = verbose ? std::atoi(verbose) : 0;
    o.cancel = cancellable ? &j.cancel : nullptr;
    if (o.precision != MBL_F64 && o.precision != MBL_MIXED && o.precision != MBL_PCG32)
      fail(MBL_EINVAL, "bad precision");
    j.evals.assign(p.nev, 0.0);
    j.resid.assign(p.nev, 0.0);
    mbl_solve_info info{};
    const mbl_status st = solve_interior(*H, sigma, p.nev, p.block, p.tol, o, j.evals.data(), evecs,
                                         ldv, j.resid.data(), &info, s);
    r.status = st;
    r.sigma = sigma;
    r.nconv = info.nconv;
    r.iters = info.iters;
    r.applies = info.applies;
    r.max_resid = info.max_resid;
  } catch (const Error& e) {
    r.status = e.status;
  } catch (...) {
    r.status = MBL_EINTERNAL;
  }
  r.seconds = std::chrono::duration<double>(clk::now() - t0).count();
}

void copy_out(const Job& j, mbl_result* out) {
  double* ev = out->evals_host;
  double* rs = out->resid_host;
  double* vd = out->evecs_dev;
  const int64_t ldv = out->ldv;
  *out = j.r;
  out->evals_host = ev;
  out->resid_host = rs;
  out->evecs_dev = vd;
  out->ldv = ldv;
  if (ev && !j.evals.empty()) std::copy(j.evals.begin(), j.evals.end(), ev);
  if (rs && !j.resid.empty()) std::copy(j.resid.begin(), j.resid.end(), rs);
}

hipStream_t new_stream() {
  hipStream_t s;
  MBL_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  return s;
}

}  // namespace

size_t solve_footprint(int L, double Sz, int b, int prec) {
  return footprint(sector_dim(L, Sz), b, prec);
}

mbl_status batch_solve(int count, const mbl_problem* probs, mbl_result* res, int conc) {
  int dev = 0;
  MBL_HIP(hipGetDevice(&dev));
  std::vector<std::unique_ptr<Job>> jobs(count);
  for (int i = 0; i < count; ++i) {
    jobs[i] = std::make_unique<Job>();
    jobs[i]->p = probs[i];
    if (probs[i].h_host && probs[i].L > 0 && probs[i].L <= kMaxL)
      jobs[i]->h.assign(probs[i].h_host, probs[i].h_host + probs[i].L);
    else
      jobs[i]->h.assign(std::max(0, std::min(probs[i].L, kMaxL)), NAN);
  }
  // With the fused CG (MBL_BATCH_FUSE=1; off by default: measured no faster
  // than concurrent streams on the batched workload, slower with longer
  // gather windows) the workers take the problems in order of chain length
  // and block shape, so that the solves running side by side share their CG
  // launches; results go to each problem's own slot either way.
  const char* fe = std::getenv("MBL_BATCH_FUSE");
  const bool fuse = fe != nullptr && std::atoi(fe) != 0 && conc > 1 && count > 1;
  const char* we = std::getenv("MBL_FUSE_WAIT_MS");
  std::unique_ptr<CgFuser, void (*)(CgFuser*)> fuser(
      fuse ? cg_fuser_create(std::min(conc, 8), we ? std::atof(we) : 0.5) : nullptr,
      cg_fuser_destroy);
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  if (fuse)
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      const mbl_problem &x = probs[a], &y = probs[b];
      return std::make_tuple(x.L, x.Sz, x.block, x.precision, x.pcg_iters) <
             std::make_tuple(y.L, y.Sz, y.block, y.precision, y.pcg_iters);
    });
  const auto t0 = clk::now();
  std::atomic<int> next{0};
  auto worker = [&]() {
    (void)hipSetDevice(dev);
    hipStream_t s = nullptr;
    try {
      s = new_stream();
    } catch (...) {
      return;
    }
    t_cg_fuser = fuser.get();
    for (int k; (k = next.fetch_add(1)) < count;) {
      const int i = order[k];
      run_problem(*jobs[i], res[i].evecs_dev, res[i].ldv, s, false);
      jobs[i]->r.latency = std::chrono::duration<double>(clk::now() - t0).count();
      copy_out(*jobs[i], &res[i]);
      jobs[i]->done = true;
    }
    t_cg_fuser = nullptr;
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  };
  std::vector<std::thread> pool;
  const int nt = std::max(1, std::min(conc, count));
  for (int t = 0; t < nt; ++t) pool.emplace_back(worker);
  for (auto& t : pool) t.join();
  if (fuser && std::getenv("MBL_FUSE_STATS")) {
    int64_t groups = 0, calls = 0;
    cg_fuser_stats(fuser.get(), &groups, &calls);
    std::fprintf(stderr, "[mbl batch] fused CG: %lld groups, %lld calls\n", (long long)groups,
                 (long long)calls);
  }
  // a problem no worker reached (every worker failed to create its stream)
  for (int i = 0; i < count; ++i)
    if (!jobs[i]->done) res[i].status = MBL_EDEVICE;
  mbl_status first = MBL_OK;
  for (int i = 0; i < count && first == MBL_OK; ++i)
    if (res[i].status != MBL_OK) first = (mbl_status)res[i].status;
  return first;
}

// ---------------------------------------------------------------------------
struct Server {
  int dev = 0;
  size_t budget = 0, in_use = 0, peak = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job*> pending;
  std::map<uint64_t, std::unique_ptr<Job>> jobs;
  std::vector<double> latencies;
  double pairs_done = 0;
  int64_t submitted = 0, admitted = 0, completed = 0, rejected = 0, running = 0;
  uint64_t next_ticket = 1;
  bool stop = false;
  clk::time_point created = clk::now();
  std::vector<std::thread> workers;
  // copies of results to the caller: a stream of its own, never the legacy
  // stream, which would have to wait for the workers' captured CG steps
  hipStream_t copy = nullptr;

  void worker_loop() {
    (void)hipSetDevice(dev);
    hipStream_t s = nullptr;
    try {
      s = new_stream();
    } catch (...) {
      return;
    }
    for (;;) {
      Job* j = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] {
          return stop || (!pending.empty() && in_use + pending.front()->fp <= budget);
        });
        if (pending.empty() || in_use + pending.front()->fp > budget) {
          if (stop && pending.empty()) break;
          continue;
        }
        j = pending.front();
        pending.pop_front();
        in_use += j->fp;
        peak = std::max(peak, in_use);
        ++admitted;
        ++running;
      }
      double* vec = nullptr;
      if (j->p.want_vectors) {
        try {
          const int64_t n = sector_dim(j->p.L, j->p.Sz);
          // freed on the copy stream once wait() has copied it out
          j->V.reset_ordered((size_t)n * std::max(1, j->p.nev) * sizeof(double), s, copy);
          vec = j->V.as<double>();
        } catch (const Error& e) {
          j->r.status = e.status;
        }
      }
      if (j->r.status == MBL_OK) run_problem(*j, vec, std::max(1, j->p.nev), s, true);
      {
        std::lock_guard<std::mutex> lk(mu);
        j->r.latency = std::chrono::duration<double>(clk::now() - j->submitted).count();
        j->done = true;
        in_use -= j->fp;
        --running;
        ++completed;
        latencies.push_back(j->r.latency);
        pairs_done += j->r.nconv;
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
};

mbl_status server_create(int device, int conc, size_t budget, Server** out) {
  auto srv = std::make_unique<Server>();
  srv->dev = device;
  MBL_HIP(hipSetDevice(device));
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    MBL_HIP(hipMemGetInfo(&fr, &tot));
    budget = (size_t)(0.9 * (double)fr);
  }
  srv->budget = budget;
  srv->copy = new_stream();
  Server* raw = srv.get();
  for (int t = 0; t < std::max(1, conc); ++t) raw->workers.emplace_back([raw] { raw->worker_loop(); });
  *out = srv.release();
  return MBL_OK;
}

mbl_status server_submit(Server* srv, const mbl_problem* rq, uint64_t* ticket) {
  auto j = std::make_unique<Job>();
  j->p = *rq;
  if (!(rq->L >= 2 && rq->L <= kMaxL)) fail(MBL_EINVAL, "L must be in [2, 32]");
  if (!rq->h_host) fail(MBL_EINVAL, "h is NULL");
  j->h.assign(rq->h_host, rq->h_host + rq->L);
  j->p.h_host = nullptr;
  if (rq->block < 1 || rq->block > 320 || rq->nev < 1 || rq->nev > rq->block)
    fail(MBL_EINVAL, "need 1 <= nev <= block <= 320");
  j->fp = footprint(sector_dim(rq->L, rq->Sz), rq->block, rq->precision) +
          (rq->want_vectors ? (size_t)sector_dim(rq->L, rq->Sz) * rq->nev * sizeof(double) : 0);
  j->submitted = clk::now();
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->stop) fail(MBL_EINVAL, "server is stopping");
  ++srv->submitted;
  if (j->fp > srv->budget) {
    ++srv->rejected;
    fail(MBL_ENOMEM, "request footprint " + std::to_string(j->fp) + " B exceeds the budget " +
                         std::to_string(srv->budget) + " B");
  }
  j->ticket = srv->next_ticket++;
  *ticket = j->ticket;
  srv->pending.push_back(j.get());
  srv->jobs[j->ticket] = std::move(j);
  srv->cv_work.notify_all();
  return MBL_OK;
}

mbl_status server_wait(Server* srv, uint64_t ticket, double timeout_s, mbl_result* out) {
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->jobs.find(ticket);
  if (it == srv->jobs.end()) fail(MBL_EINVAL, "unknown ticket");
  Job* j = it->second.get();
  auto ready = [&] { return j->done; };
  if (timeout_s < 0) {
    srv->cv_done.wait(lk, ready);
  } else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
    return MBL_ETIMEOUT;
  }
  copy_out(*j, out);
  // take the job out of the table, then copy its vectors without holding the
  // lock (workers finishing other jobs need it)
  std::unique_ptr<Job> own = std::move(it->second);
  srv->jobs.erase(it);
  lk.unlock();
  if (out->evecs_dev && own->V.get() && own->n > 0) {
    MBL_HIP(hipMemcpy2DAsync(out->evecs_dev, out->ldv * sizeof(double), own->V.get(),
                             own->p.nev * sizeof(double), own->p.nev * sizeof(double), own->n,
                             hipMemcpyDeviceToDevice, srv->copy));
    MBL_HIP(hipStreamSynchronize(srv->copy));
  }
  return MBL_OK;
}

mbl_status server_cancel(Server* srv, uint64_t ticket) {
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(ticket);
    if (it == srv->jobs.end() || it->second->done) fail(MBL_EINVAL, "unknown or finished ticket");
    Job* j = it->second.get();
    auto q = std::find(srv->pending.begin(), srv->pending.end(), j);
    if (q == srv->pending.end()) {
      j->cancel = 1;  // running: the solve stops at its next check
      return MBL_OK;
    }
    srv->pending.erase(q);
    j->r.status = MBL_ECANCELLED;
    j->r.latency = std::chrono::duration<double>(clk::now() - j->submitted).count();
    j->done = true;
    ++srv->completed;
  }
  srv->cv_done.notify_all();
  srv->cv_work.notify_all();
  return MBL_OK;
}

mbl_status server_stats(Server* srv, mbl_server_stats* st) {
  std::lock_guard<std::mutex> lk(srv->mu);
  st->submitted = srv->submitted;
  st->admitted = srv->admitted;
  st->completed = srv->completed;
  st->rejected = srv->rejected;
  st->in_flight = srv->running;
  std::vector<double> l = srv->latencies;
  std::sort(l.begin(), l.end());
  auto pct = [&](double q) {
    if (l.empty()) return 0.0;
    const size_t k = (size_t)std::min<double>((double)l.size() - 1, std::ceil(q * l.size()) - 1);
    return l[k];
  };
  st->p50_latency = pct(0.50);
  st->p99_latency = pct(0.99);
  const double el = std::chrono::duration<double>(clk::now() - srv->created).count();
  st->throughput_pairs = el > 0 ? srv->pairs_done / el : 0.0;
  st->budget_bytes = srv->budget;
  st->peak_bytes = srv->peak;
  return MBL_OK;
}

void server_destroy(Server* srv) {
  {
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_done.wait(lk, [&] { return srv->pending.empty() && srv->running == 0; });
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  for (auto& t : srv->workers) t.join();
  srv->jobs.clear();  // results never waited for: their vectors free on `copy`
  if (srv->copy) {
    (void)hipStreamSynchronize(srv->copy);
    (void)hipStreamDestroy(srv->copy);
  }
  delete srv;
}

}  // namespace mbl
