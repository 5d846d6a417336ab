"""Host logic of the split apply: the far-bond pass's row segments.

The segment builder (paper_2012_00217_amd/csrc/split_plan.h) is plain C++; this
test compiles it with g++ into a small driver that enumerates the sector by
brute force and checks, for several (L, k, m, chunk):
  * every row is covered by exactly one segment;
  * every far-bond (i >= m) flip-flop target of a row lies in the same
    (kl, chunk) group as the row, so one group is self-contained.
"""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HDR = os.path.join(os.path.dirname(HERE), "paper_2012_00217_amd", "csrc", "split_plan.h")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include "split_plan.h"
int main(int argc, char** argv) {
  const int L = atoi(argv[1]), k = atoi(argv[2]), m = atoi(argv[3]), chunk = atoi(argv[4]);
  static uint32_t C[33 * 33];
  for (int i = 0; i < 33; ++i) {
    C[i * 33] = 1;
    for (int t = 1; t <= i; ++t) C[i * 33 + t] = C[(i - 1) * 33 + t - 1] + (t <= i - 1 ? C[(i - 1) * 33 + t] : 0);
  }
  std::vector<uint64_t> st;
  for (uint64_t s = 0; s < (1ull << L); ++s) if (__builtin_popcountll(s) == k) st.push_back(s);
  const int64_t n = (int64_t)st.size();
  std::vector<int64_t> start; std::vector<int> len;
  mbl::split_segments(L, k, m, chunk, C, 33, start, len);
  // group of a segment: consecutive segments with the same (kl, chunk); a new
  // group starts whenever the row offset within its hi run changes
  std::vector<int64_t> group(n, -1), cover(n, 0);
  int64_t g = -1, prev_off = -1, prev_kl = -1;
  for (size_t j = 0; j < start.size(); ++j) {
    const uint64_t s0 = st[start[j]];
    const int kl = __builtin_popcountll(s0 & ((1ull << m) - 1));
    // offset of the segment's first row within its hi run
    const uint64_t hi = s0 >> m;
    const int64_t run0 = std::lower_bound(st.begin(), st.end(), hi << m) - st.begin();
    const int64_t off = start[j] - run0;
    if (off != prev_off || kl != prev_kl) { ++g; prev_off = off; prev_kl = kl; }
    if (len[j] <= 0 || len[j] > chunk) { printf("bad length\n"); return 1; }
    for (int r = 0; r < len[j]; ++r) {
      const int64_t row = start[j] + r;
      if (row < 0 || row >= n) { printf("row out of range\n"); return 1; }
      if ((st[row] >> m) != hi) { printf("segment crosses a hi run\n"); return 1; }
      cover[row]++; group[row] = g;
    }
  }
  for (int64_t r = 0; r < n; ++r) if (cover[r] != 1) { printf("row %lld covered %lld times\n", (long long)r, (long long)cover[r]); return 1; }
  for (int64_t r = 0; r < n; ++r)
    for (int i = m; i < L - 1; ++i) {
      const uint64_t s = st[r];
      if (((s >> i) & 1) == ((s >> (i + 1)) & 1)) continue;
      const uint64_t t = s ^ (3ull << i);
      const int64_t rt = std::lower_bound(st.begin(), st.end(), t) - st.begin();
      if (group[rt] != group[r]) { printf("far bond %d of row %lld leaves its group\n", i, (long long)r); return 1; }
    }
  printf("ok %lld rows %zu segments %lld groups\n", (long long)n, start.size(), (long long)(g + 1));
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("split")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    exe = d / "driver"
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", os.path.dirname(HDR), str(src), "-o", str(exe)],
                   check=True)
    return str(exe)


@pytest.mark.parametrize("L,k,m,chunk", [(12, 6, 7, 8), (14, 7, 9, 32), (13, 5, 6, 5), (16, 8, 11, 32),
                                         (16, 3, 12, 16), (18, 9, 13, 64), (10, 5, 1, 4)])
def test_segments_cover_rows_once_and_keep_far_bonds_inside(driver, L, k, m, chunk):
    out = subprocess.run([driver, str(L), str(k), str(m), str(chunk)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok")
