// Row segments of the far-bond pass of the split apply (host code, no HIP).
//
// Write a sector state as s = hi * 2^m + lo (lo: sites 0..m-1).  A flip-flop
// on a bond i >= m changes only hi, so it maps the row of (hi, lo) to the row
// of (hi', lo): same lo, same number kl of up spins in lo.  In the ascending
// row order, the rows of one hi form a contiguous run that lists the lo
// patterns with kl up spins in the same order for every hi.  Cutting those
// runs into chunks of `chunk` consecutive lo positions and listing, chunk by
// chunk, the piece of every hi gives segments such that all far-bond targets
// of a segment's rows lie in segments of the same chunk.  Processed in that
// order, a chunk's rows are fetched once and reused by all its far bonds.
#pragma once

#include <cstdint>
#include <vector>

namespace mbl {

// C: Pascal table, C[i * ldc + t] = binomial(i, t).  k: up spins of the
// sector.  Appends, for every kl, chunk and hi (in that nesting order), the
// first row and the row count of one segment.
inline void split_segments(int L, int k, int m, int chunk, const uint32_t* C, int ldc,
                           std::vector<int64_t>& start, std::vector<int>& len) {
  start.clear();
  len.clear();
  if (m <= 0 || m >= L || chunk <= 0) return;
  const int nh = L - m;
  auto binom = [&](int i, int t) -> int64_t {
    return (t < 0 || t > i) ? 0 : (int64_t)C[i * ldc + t];
  };
  // colex rank of a state: sum over its up spins p_0 < p_1 < ... of C(p_t, t+1)
  auto rank = [&](uint64_t s) -> int64_t {
    int64_t r = 0;
    int t = 0;
    for (int p = 0; p < L; ++p)
      if ((s >> p) & 1u) r += binom(p, ++t);
    return r;
  };
  for (int kl = 0; kl <= m && kl <= k; ++kl) {
    const int kh = k - kl;
    if (kh > nh) continue;
    const int64_t nlo = binom(m, kl);
    std::vector<uint32_t> his;
    for (uint32_t hi = 0; hi < (1u << nh); ++hi)
      if (__builtin_popcount(hi) == kh) his.push_back(hi);
    if (his.empty() || nlo == 0) continue;
    const uint64_t lomin = (kl == 0) ? 0 : ((1ull << kl) - 1);
    std::vector<int64_t> base(his.size());
    for (size_t j = 0; j < his.size(); ++j) base[j] = rank(((uint64_t)his[j] << m) | lomin);
    for (int64_t c0 = 0; c0 < nlo; c0 += chunk) {
      const int l = (int)((nlo - c0) < chunk ? (nlo - c0) : chunk);
      for (size_t j = 0; j < his.size(); ++j) {
        start.push_back(base[j] + c0);
        len.push_back(l);
      }
    }
  }
}

}  // namespace mbl
