// MBL observables of computed eigenpairs (paper Sec. 2.2) and spectrum
// slicing (Sec. 3.1, third level of concurrency: eigenvalue chunks).
//
// Entanglement entropy across the cut between sites l-1 and l.  Write a
// sector state as s = u 2^l + v (u: right part, sites l..L-1; v: left part).
// The reduced density matrix of the left part is block diagonal in the number
// of up spins kA of v; its block is M M^T with M[v][u] = psi(s).  In the
// ascending (colex) row order the rows with one fixed u are consecutive and
// list the admissible v in the same order for every u, so column u of M is a
// contiguous segment of psi starting at the row of (u, lowest v).  Each block
// is therefore a Gram matrix of contiguous segments (or of their transposes,
// whichever dimension is smaller); its eigenvalues p give
// S = -sum p ln p.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>

#include "common.h"

namespace mbl {
namespace {

// G (dim x dim) from segments of psi (column j of a row-major block, stride
// ld): by_rows -> G[i][k] = sum_u psi[st[u]+i] psi[st[u]+k] (dim = a, sum over
// c segments); else G[u1][u2] = sum_v psi[st[u1]+v] psi[st[u2]+v] (dim = c).
__global__ __launch_bounds__(256) void k_seg_gram(const double* __restrict__ psi, int64_t ld,
                                                  const int64_t* __restrict__ st, int c, int a,
                                                  int by_rows, double* __restrict__ G) {
  const int dim = by_rows ? a : c;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)dim * dim) return;
  const int i = (int)(e / dim), k = (int)(e % dim);
  double s = 0.0;
  if (by_rows) {
    for (int u = 0; u < c; ++u) s += psi[(st[u] + i) * ld] * psi[(st[u] + k) * ld];
  } else {
    for (int v = 0; v < a; ++v) s += psi[(st[i] + v) * ld] * psi[(st[k] + v) * ld];
  }
  G[e] = s;
}

int64_t binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  int64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

}  // namespace

void entanglement_entropy(const Ham& H, const double* V, int64_t ldv, int nev, int cut, double* S,
                          hipStream_t s) {
  const int L = H.L, k = H.nup, R = L - cut;
  std::vector<double> ent(nev, 0.0);
  for (int kA = std::max(0, k - R); kA <= std::min(cut, k); ++kA) {
    const int a = (int)binom(cut, kA), c = (int)binom(R, k - kA);
    if (a == 0 || c == 0) continue;
    // first row of every right-part pattern u (popcount k - kA), in order
    uint64_t vmin = (kA == 0) ? 0 : ((1ull << kA) - 1);
    std::vector<uint64_t> q;
    q.reserve(c);
    for (uint64_t u = 0; u < (1ull << R); ++u)
      if (__builtin_popcountll(u) == k - kA) q.push_back((u << cut) | vmin);
    DevBuf qd(q.size() * sizeof(uint64_t), s), st(q.size() * sizeof(int64_t), s);
    MBL_HIP(hipMemcpyAsync(qd.get(), q.data(), qd.bytes(), hipMemcpyHostToDevice, s));
    rank_states(H, qd.as<uint64_t>(), (int64_t)q.size(), st.as<int64_t>(), s);
    const bool by_rows = a <= c;
    const int dim = by_rows ? a : c;
    DevBuf G((size_t)dim * dim * sizeof(double), s), w((size_t)dim * sizeof(double), s),
        Z((size_t)dim * dim * sizeof(double), s), work(small_eigh_work_bytes(dim), s);
    std::vector<double> p(dim);
    for (int j = 0; j < nev; ++j) {
      hipLaunchKernelGGL(k_seg_gram, dim3((unsigned)(((int64_t)dim * dim + 255) / 256)), dim3(256),
                         0, s, V + j, ldv, st.as<int64_t>(), c, a, (int)by_rows, G.as<double>());
      MBL_CHECK_LAUNCH();
      // only the eigenvalues are needed: blocks up to 128 take the values-only path
      double* zv = dim + (dim & 1) <= 128 ? nullptr : Z.as<double>();
      small_eigh(dim, G.as<double>(), dim, w.as<double>(), zv, dim, work.as<double>(), s);
      MBL_HIP(hipMemcpyAsync(p.data(), w.get(), dim * sizeof(double), hipMemcpyDeviceToHost, s));
      MBL_HIP(hipStreamSynchronize(s));
      for (double x : p)
        if (x > 1e-300) ent[j] -= x * std::log(x);
    }
  }
  for (int j = 0; j < nev; ++j) S[j] = ent[j];
}

double mean_gap_ratio(const double* e, int count) {
  std::vector<double> v(e, e + count);
  std::sort(v.begin(), v.end());
  double sum = 0;
  int m = 0;
  for (int i = 0; i + 2 < count; ++i) {
    const double d1 = v[i + 1] - v[i], d2 = v[i + 2] - v[i + 1];
    const double hi = std::max(d1, d2);
    if (hi > 0) {
      sum += std::min(d1, d2) / hi;
      ++m;
    }
  }
  return m ? sum / m : NAN;
}

// Several shifts of one Hamiltonian, `conc` at a time on worker streams that
// share the handle's read-only tables.
mbl_status solve_slices(const Ham& H, int count, const double* sigmas, int nev, int b, double tol,
                        const mbl_solve_opts& o, double* evals, double* resid, int conc) {
  int dev = 0;
  MBL_HIP(hipGetDevice(&dev));
  std::atomic<int> next{0};
  std::vector<mbl_status> st(count, MBL_EINTERNAL);
  auto worker = [&]() {
    (void)hipSetDevice(dev);
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
    for (int i; (i = next.fetch_add(1)) < count;) {
      try {
        st[i] = solve_interior(H, sigmas[i], nev, b, tol, o, evals + (size_t)i * nev, nullptr, 0,
                               resid ? resid + (size_t)i * nev : nullptr, nullptr, s);
      } catch (const Error& e) {
        st[i] = e.status;
      } catch (...) {
        st[i] = MBL_EINTERNAL;
      }
    }
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  };
  std::vector<std::thread> pool;
  for (int t = 0; t < std::max(1, std::min(conc, count)); ++t) pool.emplace_back(worker);
  for (auto& t : pool) t.join();
  for (auto x : st)
    if (x != MBL_OK) return x;
  return MBL_OK;
}

}  // namespace mbl
