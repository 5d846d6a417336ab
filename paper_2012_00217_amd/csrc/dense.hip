// Small dense FP64 linear algebra of LOBPCG's Rayleigh-Ritz and
// orthonormalisation steps (paper Sec. 3.2), sizes up to a few hundred.
//
//  * Symmetric eigendecomposition by cyclic two-sided Jacobi with the
//    round-robin (tournament) pair ordering: in each round the indices are
//    split into disjoint pairs, so all rotations of a round commute and the
//    matrix splits into 2 x 2 blocks that are updated independently,
//    A_kl <- J_k^T A_kl J_l.  Sizes <= 96 run in one workgroup with A and V in
//    LDS (<= 128 when only eigenvalues are wanted, with A alone in LDS); larger
//    ones run one kernel per round, ping-ponging A between two
//    buffers so the rotations of a round are computed from the unmodified
//    matrix.  A sweep ends with a count of rotations; none means converged.
//    Jacobi keeps small eigenvalues of positive semi-definite matrices to
//    high relative accuracy, which matters for the spectral fold.
//  * Cholesky with column dropping, R^T R = G, for Cholesky-QR: a column whose
//    pivot falls below tol * G_jj is linearly dependent on the earlier ones and
//    is dropped; the inverse of R on the kept columns is returned compacted.
//  * Small matrix products and the nearest-shift selection.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace mbl {
namespace {

constexpr double kRotTol = 1e-15;  // rotate when |a_pq| > tol * sqrt(|a_pp a_qq|)

__device__ inline void pair_of(int mm, int round, int k, int* p, int* q) {
  int a, b;
  if (k == 0) {
    a = mm - 1;
    b = round;
  } else {
    a = (round + k) % (mm - 1);
    b = (round - k + mm - 1) % (mm - 1);
  }
  *p = min(a, b);
  *q = max(a, b);
}

// Rotation (c, s) that annihilates a_pq:  A' = J^T A J with J_pp = J_qq = c,
// J_pq = s, J_qp = -s.  Returns false (c = 1, s = 0) when a_pq is negligible.
__device__ inline bool rotation(double app, double aqq, double apq, double* c, double* s) {
  if (apq == 0.0 || fabs(apq) <= kRotTol * sqrt(fabs(app * aqq))) {
    *c = 1.0;
    *s = 0.0;
    return false;
  }
  const double tau = (aqq - app) / (2.0 * apq);
  const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  *c = 1.0 / sqrt(1.0 + t * t);
  *s = t * (*c);
  return true;
}

// 2 x 2 block update B' = J_k^T B J_l.
__device__ inline void rot_block(double ck, double sk, double cl, double sl, double& bpp,
                                 double& bpq, double& bqp, double& bqq) {
  const double rpp = ck * bpp - sk * bqp, rpq = ck * bpq - sk * bqq;
  const double rqp = sk * bpp + ck * bqp, rqq = sk * bpq + ck * bqq;
  bpp = cl * rpp - sl * rpq;
  bpq = sl * rpp + cl * rpq;
  bqp = cl * rqp - sl * rqq;
  bqq = sl * rqp + cl * rqq;
}

// Whole Jacobi eigensolver in one workgroup (mm even): A and V in LDS for
// mm <= 96, or A alone when only eigenvalues are wanted (kVec false, mm <= 128).
// The pairs of a round are tabulated once per round, and every thread keeps a
// fixed pair column l (and walks rows k, or matrix rows i, with a fixed stride),
// so the inner loops do no integer division.
constexpr int kLdsPairs = 64;  // pairs per round, mm / 2 <= 64
template <bool kVec>
__global__ __launch_bounds__(1024) void k_jacobi_lds(int m, const double* __restrict__ A,
                                                     int64_t lda, double* __restrict__ w,
                                                     double* __restrict__ V, int64_t ldv,
                                                     int max_sweeps) {
  extern __shared__ double sh[];
  const int mm = m + (m & 1);
  double* a = sh;             // mm x mm
  double* v = sh + mm * mm;   // mm x mm (kVec only)
  __shared__ double cs_c[kLdsPairs], cs_s[kLdsPairs];
  __shared__ int pp[kLdsPairs], qq[kLdsPairs];
  __shared__ int nrot;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < mm * mm; e += nt) {
    const int i = e / mm, j = e % mm;
    a[e] = (i < m && j < m) ? A[(int64_t)i * lda + j] : 0.0;
    if constexpr (kVec) v[e] = (i == j) ? 1.0 : 0.0;
  }
  // symmetrise from the upper triangle
  __syncthreads();
  for (int e = tid; e < mm * mm; e += nt) {
    const int i = e / mm, j = e % mm;
    if (i > j) a[e] = a[j * mm + i];
  }
  __syncthreads();
  const int np = mm / 2;
  const int rows_per_pass = nt / np;          // threads sharing one pair column
  const int l = tid % np, r0 = tid / np;      // this thread's column and first row
  const bool worker = r0 < rows_per_pass;     // the last nt % np threads idle
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (tid == 0) nrot = 0;
    __syncthreads();
    for (int round = 0; round < mm - 1; ++round) {
      if (tid < np) {
        int p, q;
        pair_of(mm, round, tid, &p, &q);
        double c, s;
        if (rotation(a[p * mm + p], a[q * mm + q], a[p * mm + q], &c, &s)) atomicAdd(&nrot, 1);
        cs_c[tid] = c;
        cs_s[tid] = s;
        pp[tid] = p;
        qq[tid] = q;
      }
      __syncthreads();
      if (worker) {
        const int pl = pp[l], ql = qq[l];
        const double cl = cs_c[l], sl = cs_s[l];
        for (int k = r0; k < np; k += rows_per_pass) {
          const int pk = pp[k], qk = qq[k];
          double bpp = a[pk * mm + pl], bpq = a[pk * mm + ql], bqp = a[qk * mm + pl],
                 bqq = a[qk * mm + ql];
          rot_block(cs_c[k], cs_s[k], cl, sl, bpp, bpq, bqp, bqq);
          if (k == l) {
            bpq = 0.0;
            bqp = 0.0;
          }
          a[pk * mm + pl] = bpp;
          a[pk * mm + ql] = bpq;
          a[qk * mm + pl] = bqp;
          a[qk * mm + ql] = bqq;
        }
        if constexpr (kVec) {
          for (int i = r0; i < mm; i += rows_per_pass) {
            const double vp = v[i * mm + pl], vq = v[i * mm + ql];
            v[i * mm + pl] = cl * vp - sl * vq;
            v[i * mm + ql] = sl * vp + cl * vq;
          }
        }
      }
      __syncthreads();
    }
    const bool done = (nrot == 0);
    __syncthreads();
    if (done) break;
  }
  // ascending order (ties by index); padded index mm-1 (if any) is skipped
  for (int j = tid; j < m; j += nt) {
    const double dj = a[j * mm + j];
    int r = 0;
    for (int i = 0; i < m; ++i) {
      const double di = a[i * mm + i];
      r += (di < dj) || (di == dj && i < j);
    }
    w[r] = dj;
    if constexpr (kVec)
      for (int i = 0; i < m; ++i) V[(int64_t)i * ldv + r] = v[i * mm + j];
  }
}

// Multi-kernel Jacobi: one launch per round.
__global__ __launch_bounds__(256) void k_jacobi_round(int mm, int round,
                                                      const double* __restrict__ ain,
                                                      double* __restrict__ aout,
                                                      double* __restrict__ v,
                                                      int* __restrict__ nrot) {
  const int np = mm / 2;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nblk = (int64_t)np * np;
  if (e < nblk) {
    const int k = (int)(e / np), l = (int)(e % np);
    int pk, qk, pl, ql;
    pair_of(mm, round, k, &pk, &qk);
    pair_of(mm, round, l, &pl, &ql);
    double ck, sk, cl, sl;
    const bool rk = rotation(ain[pk * mm + pk], ain[qk * mm + qk], ain[pk * mm + qk], &ck, &sk);
    rotation(ain[pl * mm + pl], ain[ql * mm + ql], ain[pl * mm + ql], &cl, &sl);
    if (k == l && rk) atomicAdd(nrot, 1);
    double bpp = ain[pk * mm + pl], bpq = ain[pk * mm + ql], bqp = ain[qk * mm + pl],
           bqq = ain[qk * mm + ql];
    rot_block(ck, sk, cl, sl, bpp, bpq, bqp, bqq);
    if (k == l) {
      bpq = 0.0;
      bqp = 0.0;
    }
    aout[pk * mm + pl] = bpp;
    aout[pk * mm + ql] = bpq;
    aout[qk * mm + pl] = bqp;
    aout[qk * mm + ql] = bqq;
  } else if (e < nblk + (int64_t)mm * np) {
    const int64_t f = e - nblk;
    const int i = (int)(f / np), l = (int)(f % np);
    int pl, ql;
    pair_of(mm, round, l, &pl, &ql);
    double cl, sl;
    rotation(ain[pl * mm + pl], ain[ql * mm + ql], ain[pl * mm + ql], &cl, &sl);
    const double vp = v[i * mm + pl], vq = v[i * mm + ql];
    v[i * mm + pl] = cl * vp - sl * vq;
    v[i * mm + ql] = sl * vp + cl * vq;
  }
}

__global__ __launch_bounds__(256) void k_jacobi_init(int m, int mm, const double* __restrict__ A,
                                                     int64_t lda, double* __restrict__ a,
                                                     double* __restrict__ v) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)mm * mm) return;
  const int i = (int)(e / mm), j = (int)(e % mm);
  const int u = min(i, j), x = max(i, j);  // symmetrise from the upper triangle
  a[e] = (x < m) ? A[(int64_t)u * lda + x] : 0.0;
  v[e] = (i == j) ? 1.0 : 0.0;
}

__global__ __launch_bounds__(256) void k_jacobi_sort(int m, int mm, const double* __restrict__ a,
                                                     const double* __restrict__ v,
                                                     double* __restrict__ w,
                                                     double* __restrict__ V, int64_t ldv) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const double dj = a[(int64_t)j * mm + j];
  int r = 0;
  for (int i = 0; i < m; ++i) {
    const double di = a[(int64_t)i * mm + i];
    r += (di < dj) || (di == dj && i < j);
  }
  w[r] = dj;
  for (int i = 0; i < m; ++i) V[(int64_t)i * ldv + r] = v[(int64_t)i * mm + j];
}

// Cholesky with dropping (row-oriented) and inverse of R on the kept columns.
// G: b x b (upper triangle read).  Outputs Rinv_c (b x b, ld b; column jc is
// the jc-th kept column of R^-1, other columns zero) and *count.  R and R^-1
// live in LDS when in_lds (b <= kCholLds), else in global memory (R in the
// work buffer).  R^-1 is built one row at a time from the bottom, every
// thread owning columns, so each step is parallel over the columns.
constexpr int kCholLds = 88;  // 2 b^2 doubles + the static arrays fit 160 KB of LDS

__global__ __launch_bounds__(1024) void k_chol_drop(int b, const double* __restrict__ G,
                                                    int64_t ldg, double tol, int in_lds,
                                                    double* __restrict__ Rg,
                                                    double* __restrict__ Rinv,
                                                    int* __restrict__ count) {
  extern __shared__ double shm[];
  __shared__ int keep[1024];
  __shared__ int pos[1024];
  __shared__ double row[1024];
  __shared__ double rjj;
  const int tid = threadIdx.x, nt = blockDim.x;
  double* R = in_lds ? shm : Rg;
  double* Ri = in_lds ? shm + b * b : Rinv;
  for (int e = tid; e < b * b; e += nt) {
    R[e] = 0.0;
    Ri[e] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j < b; ++j) {
    for (int l = j + tid; l < b; l += nt) {
      double g = G[(int64_t)j * ldg + l];
      for (int k = 0; k < j; ++k)
        if (keep[k]) g -= R[k * b + j] * R[k * b + l];
      row[l] = g;
    }
    __syncthreads();
    if (tid == 0) {
      const double gjj = G[(int64_t)j * ldg + j];
      const double d = row[j];
      keep[j] = (gjj > 0.0) && (d > tol * gjj) && isfinite(d);
      rjj = keep[j] ? sqrt(d) : 0.0;
    }
    __syncthreads();
    if (keep[j])
      for (int l = j + tid; l < b; l += nt) R[j * b + l] = row[l] / rjj;
    __syncthreads();
  }
  if (tid == 0) {
    int c = 0;
    for (int j = 0; j < b; ++j) {
      pos[j] = c;
      c += keep[j];
    }
    *count = c;
  }
  __syncthreads();
  // row i of R^-1 (kept columns only) from the rows below it
  for (int i = b - 1; i >= 0; --i) {
    if (keep[i]) {
      const double rii = R[i * b + i];
      for (int j = i + tid; j < b; j += nt) {
        if (!keep[j]) continue;
        const int jc = pos[j];
        if (j == i) {
          Ri[i * b + jc] = 1.0 / rii;
          continue;
        }
        double s = 0.0;
        for (int k = i + 1; k <= j; ++k)
          if (keep[k]) s += R[i * b + k] * Ri[k * b + jc];
        Ri[i * b + jc] = -s / rii;
      }
    }
    __syncthreads();
  }
  if (in_lds)
    for (int e = tid; e < b * b; e += nt) Rinv[e] = Ri[e];
}

// C = alpha op(A) op(B) + beta C for small row-major FP64 matrices.
__global__ __launch_bounds__(256) void k_small_gemm(int M, int N, int K, double alpha,
                                                    const double* __restrict__ A, int64_t lda,
                                                    int ta, const double* __restrict__ B,
                                                    int64_t ldb, int tb, double beta,
                                                    double* __restrict__ C, int64_t ldc) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)M * N) return;
  const int i = (int)(e / N), j = (int)(e % N);
  double s = 0.0;
  for (int k = 0; k < K; ++k) {
    const double av = ta ? A[(int64_t)k * lda + i] : A[(int64_t)i * lda + k];
    const double bv = tb ? B[(int64_t)j * ldb + k] : B[(int64_t)k * ldb + j];
    s += av * bv;
  }
  C[(int64_t)i * ldc + j] = alpha * s + (beta == 0.0 ? 0.0 : beta * C[(int64_t)i * ldc + j]);
}

__global__ __launch_bounds__(256) void k_gather_cols(int rows, int nsel, const int* __restrict__ sel,
                                                     const double* __restrict__ Z, int64_t ldz,
                                                     double* __restrict__ out, int64_t ldo) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)rows * nsel) return;
  const int i = (int)(e / nsel), j = (int)(e % nsel);
  out[(int64_t)i * ldo + j] = Z[(int64_t)i * ldz + sel[j]];
}

inline unsigned g1(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

size_t small_eigh_work_bytes(int m) {
  const int64_t mm = m + (m & 1);
  return (size_t)(3 * mm * mm) * sizeof(double) + 256;
}

void small_eigh(int m, const double* A, int64_t lda, double* w, double* V, int64_t ldv,
                double* work, hipStream_t s) {
  PhaseTick tick(PhaseClock::SMALL, s);
  if (m <= 0) return;
  const int mm = m + (m & 1);
  const int max_sweeps = 30;
  if (m == 1) {
    MBL_HIP(hipMemcpyAsync(w, A, sizeof(double), hipMemcpyDeviceToDevice, s));
    if (V) {
      const double one = 1.0;
      MBL_HIP(hipMemcpyAsync(V, &one, sizeof(double), hipMemcpyHostToDevice, s));
      MBL_HIP(hipStreamSynchronize(s));
    }
    return;
  }
  if (!V && mm <= 2 * kLdsPairs) {
    // eigenvalues only: A alone in LDS
    const size_t shm = (size_t)mm * mm * sizeof(double);
    MBL_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_jacobi_lds<false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    hipLaunchKernelGGL(k_jacobi_lds<false>, dim3(1), dim3(1024), shm, s, m, A, lda, w,
                       (double*)nullptr, (int64_t)0, max_sweeps);
    MBL_CHECK_LAUNCH();
    return;
  }
  if (!V) fail(MBL_EINTERNAL, "small_eigh: eigenvectors are needed above 128");
  if (mm <= 96) {
    const size_t shm = (size_t)2 * mm * mm * sizeof(double);
    MBL_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_jacobi_lds<true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    hipLaunchKernelGGL(k_jacobi_lds<true>, dim3(1), dim3(1024), shm, s, m, A, lda, w, V, ldv,
                       max_sweeps);
    MBL_CHECK_LAUNCH();
    return;
  }
  double* a0 = work;
  double* a1 = work + (size_t)mm * mm;
  double* v = work + (size_t)2 * mm * mm;
  int* nrot = reinterpret_cast<int*>(work + (size_t)3 * mm * mm);
  hipLaunchKernelGGL(k_jacobi_init, dim3(g1((int64_t)mm * mm)), dim3(256), 0, s, m, mm, A, lda,
                     a0, v);
  MBL_CHECK_LAUNCH();
  const int np = mm / 2;
  const int64_t threads = (int64_t)np * np + (int64_t)mm * np;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    MBL_HIP(hipMemsetAsync(nrot, 0, sizeof(int), s));
    for (int round = 0; round < mm - 1; ++round) {
      hipLaunchKernelGGL(k_jacobi_round, dim3(g1(threads)), dim3(256), 0, s, mm, round, a0, a1, v,
                         nrot);
      MBL_CHECK_LAUNCH();
      std::swap(a0, a1);
    }
    int h_nrot = 0;
    MBL_HIP(hipMemcpyAsync(&h_nrot, nrot, sizeof(int), hipMemcpyDeviceToHost, s));
    MBL_HIP(hipStreamSynchronize(s));
    if (h_nrot == 0) break;
  }
  hipLaunchKernelGGL(k_jacobi_sort, dim3(g1(m)), dim3(256), 0, s, m, mm, a0, v, w, V, ldv);
  MBL_CHECK_LAUNCH();
}

// Cholesky-with-dropping of a b x b Gram; returns the number of kept columns.
int chol_drop(int b, const double* G, int64_t ldg, double tol, double* Rinv, double* work,
              int* dcount, hipStream_t s) {
  PhaseTick tick(PhaseClock::SMALL, s);
  if (b <= 0) return 0;
  if (b > 1024) fail(MBL_EINVAL, "chol_drop: b > 1024");
  const int in_lds = b <= kCholLds;
  const size_t shm = in_lds ? (size_t)2 * b * b * sizeof(double) : 0;
  if (in_lds)
    MBL_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_chol_drop),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
  hipLaunchKernelGGL(k_chol_drop, dim3(1), dim3(1024), shm, s, b, G, ldg, tol, in_lds, work, Rinv,
                     dcount);
  MBL_CHECK_LAUNCH();
  int c = 0;
  MBL_HIP(hipMemcpyAsync(&c, dcount, sizeof(int), hipMemcpyDeviceToHost, s));
  MBL_HIP(hipStreamSynchronize(s));
  return c;
}

void small_gemm(int M, int N, int K, double alpha, const double* A, int64_t lda, bool ta,
                const double* B, int64_t ldb, bool tb, double beta, double* C, int64_t ldc,
                hipStream_t s) {
  PhaseTick tick(PhaseClock::SMALL, s);
  if ((int64_t)M * N == 0) return;
  hipLaunchKernelGGL(k_small_gemm, dim3(g1((int64_t)M * N)), dim3(256), 0, s, M, N, K, alpha, A,
                     lda, (int)ta, B, ldb, (int)tb, beta, C, ldc);
  MBL_CHECK_LAUNCH();
}


void gather_cols(int rows, int nsel, const int* sel, const double* Z, int64_t ldz, double* out,
                 int64_t ldo, hipStream_t s) {
  if ((int64_t)rows * nsel == 0) return;
  hipLaunchKernelGGL(k_gather_cols, dim3(g1((int64_t)rows * nsel)), dim3(256), 0, s, rows, nsel,
                     sel, Z, ldz, out, ldo);
  MBL_CHECK_LAUNCH();
}

}  // namespace mbl
