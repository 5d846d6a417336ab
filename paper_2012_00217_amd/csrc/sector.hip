// Sector tables of the spin chain: Pascal table, row -> state (unrank),
// state -> row (rank), the diagonal <s|H|s> and the Jacobi diagonal of the
// spectral fold.  Paper Sec. 2.1 (S^z sectors, eq. (1)/(2)) and Sec. 3.2.
//
// Row order is ascending integer value of the state.  Within a sector with k
// up spins this is the colexicographic order of the up-spin positions
// p_0 < p_1 < ... < p_{k-1}, whose rank is  sum_t C(p_t, t + 1).  A flip-flop
// on bond (i, i+1) moves one up spin by one site, so by Pascal's rule it
// shifts the rank by exactly C(i, t), t = number of up spins below site i:
// + if the up spin moves from i to i+1, - if it moves from i+1 to i.  The
// apply kernels use that identity to find every off-diagonal column in O(1).
#include "common.h"

namespace mbl {

std::vector<uint32_t> pascal_table() {
  std::vector<uint32_t> c(kPascal * kPascal, 0);
  for (int i = 0; i < kPascal; ++i) {
    c[i * kPascal] = 1;
    for (int t = 1; t <= i; ++t)
      c[i * kPascal + t] = c[(i - 1) * kPascal + t - 1] + (t <= i - 1 ? c[(i - 1) * kPascal + t] : 0);
  }
  return c;
}

namespace {

__global__ __launch_bounds__(256) void k_unrank(uint32_t* __restrict__ states, int64_t n, int L,
                                                int k, const uint32_t* __restrict__ pascal) {
  __shared__ uint32_t C[kPascal * kPascal];
  for (int i = threadIdx.x; i < kPascal * kPascal; i += blockDim.x) C[i] = pascal[i];
  __syncthreads();
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  // Greedy colex unrank: the highest up spin sits at the largest p with
  // C(p, k) <= rank; remove its contribution and repeat for k-1, ...
  uint32_t rem = (uint32_t)r, s = 0;
  int p = L - 1;
  for (int t = k; t >= 1; --t) {
    while (C[p * kPascal + t] > rem) --p;
    s |= 1u << p;
    rem -= C[p * kPascal + t];
    --p;
  }
  states[r] = s;
}

__global__ __launch_bounds__(256) void k_rank(const uint64_t* __restrict__ q, int64_t cnt,
                                              int64_t* __restrict__ out, int L, int k,
                                              const uint32_t* __restrict__ pascal) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const uint64_t s = q[i];
  if ((L < 64 && (s >> L) != 0) || __popcll(s) != k) {
    out[i] = -1;
    return;
  }
  int64_t r = 0;
  int t = 0;
  for (int p = 0; p < L; ++p)
    if ((s >> p) & 1) {
      ++t;
      r += pascal[p * kPascal + t];
    }
  out[i] = r;
}

// <s|H|s> = E_lo(lo) + E_hi(hi) + E_mid for s = (hi << q) | lo: each half's
// energy (its inner ZZ bonds, +-J Delta / 4 for aligned / anti-aligned, and
// its fields h_i (b_i - 1/2)) from a table, plus the ZZ term of the bond
// (q-1, q).  The split apply kernels evaluate the same sum in the same order.
struct DiagArgs {
  int q;
  double zz4;
  const double* Elo;
  const double* Ehi;
};

__global__ __launch_bounds__(256) void k_diag(const uint32_t* __restrict__ states, int64_t n,
                                              DiagArgs a, double* __restrict__ d64) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  const uint32_t s = states[r];
  const uint32_t lo = s & ((1u << a.q) - 1u), hi = s >> a.q;
  const bool anti = (((lo >> (a.q - 1)) ^ hi) & 1u) != 0;
  d64[r] = (a.Elo[lo] + a.Ehi[hi]) + (anti ? -a.zz4 : a.zz4);
}

// Jacobi diagonal of (H - sigma)^2: row r of H - sigma has (E - sigma) on the
// diagonal and J/2 in each of its nd off-diagonal positions.
template <class T>
__global__ __launch_bounds__(256) void k_jacobi(const uint32_t* __restrict__ states,
                                                const double* __restrict__ diag, int64_t n, int L,
                                                double sigma, double halfJ, T* __restrict__ out) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  const uint32_t s = states[r];
  const uint32_t bondmask = (L >= 2) ? ((1u << (L - 1)) - 1u) : 0u;
  const int nd = __popc((s ^ (s >> 1)) & bondmask);
  const double e = diag[r] - sigma;
  out[r] = (T)(e * e + halfJ * halfJ * (double)nd);
}

inline unsigned grid1(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void build_tables(Ham& H, hipStream_t s) {
  H.pascal_host = pascal_table();
  H.table(H.pascal, H.pascal_host.size() * sizeof(uint32_t), s);
  MBL_HIP(hipMemcpyAsync(H.pascal.get(), H.pascal_host.data(), H.pascal.bytes(),
                         hipMemcpyHostToDevice, s));
  H.table(H.states, (size_t)H.n * sizeof(uint32_t), s);
  H.table(H.diag, (size_t)H.n * sizeof(double), s);
  hipLaunchKernelGGL(k_unrank, dim3(grid1(H.n)), dim3(256), 0, s, H.states.as<uint32_t>(), H.n,
                     H.L, H.nup, H.pascal.as<uint32_t>());
  MBL_CHECK_LAUNCH();
  build_split_tables(H, s);
  if (!H.split.ok) fail(MBL_EINTERNAL, "sector tables: chain too short to split");
  DiagArgs a{};
  a.q = H.split.q;
  a.zz4 = 0.25 * H.J * H.Delta;
  a.Elo = H.split.Elo_v.as<double>();
  a.Ehi = H.split.Ehi_v.as<double>();
  hipLaunchKernelGGL(k_diag, dim3(grid1(H.n)), dim3(256), 0, s, H.states.as<uint32_t>(), H.n, a,
                     H.diag.as<double>());
  MBL_CHECK_LAUNCH();
}

void rank_states(const Ham& H, const uint64_t* q_dev, int64_t cnt, int64_t* out_dev,
                 hipStream_t s) {
  if (cnt == 0) return;
  hipLaunchKernelGGL(k_rank, dim3(grid1(cnt)), dim3(256), 0, s, q_dev, cnt, out_dev, H.L, H.nup,
                     H.pascal.as<uint32_t>());
  MBL_CHECK_LAUNCH();
}

template <class T>
void launch_jacobi(const Ham& H, double sigma, T* out, hipStream_t s) {
  hipLaunchKernelGGL(k_jacobi<T>, dim3(grid1(H.n)), dim3(256), 0, s, H.states.as<uint32_t>(),
                     H.diag.as<double>(), H.n, H.L, sigma, 0.5 * H.J, out);
  MBL_CHECK_LAUNCH();
}

template void launch_jacobi<double>(const Ham&, double, double*, hipStream_t);
template void launch_jacobi<float>(const Ham&, double, float*, hipStream_t);

}  // namespace mbl
