// Tall-skinny block kernels of LOBPCG (paper Sec. 3.2, property (ii): a block
// method turns the work into matrix-matrix operations).
//
//  * Gram products C = A^T B of n x p and n x q blocks on the matrix cores:
//    v_mfma_f64_16x16x4f64 for FP64 blocks, v_mfma_f32_16x16x4f32 with FP32
//    accumulation for FP32 blocks.  The n dimension is split over workgroups;
//    each writes an FP64 partial tile and a second kernel folds the partials
//    in split order, so the result is bitwise reproducible.
//  * Block combination Y = A C + beta Y with a small FP64 coefficient matrix
//    C (rounded to the block type), register-tiled through LDS.
//  * Precision conversion and the counter-based random starting block.
#include <algorithm>
#include <mutex>
#include <string>

#include "common.h"

namespace mbl {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <class T>
struct Mfma;
// Output row of element v held by lane group g = lane / 16 (column = lane % 16):
// the FP64 instruction interleaves the four lane groups row by row, the FP32
// one gives each lane group four consecutive rows.
template <>
struct Mfma<double> {
  using acc = d4;
  __device__ static acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int g, int v) { return g + 4 * v; }
};
template <>
struct Mfma<float> {
  using acc = f4;
  __device__ static acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int g, int v) { return 4 * g + v; }
};

// One workgroup = 4 waves = a 64 x 64 tile of C; wave (wy, wx) owns the
// 32 x 32 quadrant as 2 x 2 blocks of 16 x 16.  16 x 16 x 4 MFMA operand
// layout: lane l supplies A[i = l % 16][k = l / 16] and B[k = l / 16][j = l % 16];
// it receives D[Mfma<T>::row(l / 16, v)][l % 16], v = 0..3.  For C = A^T B the MFMA A
// operand is the transpose of the block, so both operands are 4 rows x 16
// consecutive columns of the row-major blocks.
//
// The rows are consumed in slabs of 32: the workgroup stages the slab's
// 32 x 64 panels of A and B in LDS (16-byte loads when the blocks are aligned,
// each element read from memory once per workgroup), and the next slab's
// loads are in flight while the waves run their 32 MFMAs on the current one.
// sym (A = B, p = q): only the tiles on and above the diagonal are formed;
// blockIdx.x enumerates them row by row, and a diagonal tile stages one panel.
constexpr int kSlab = 32;

template <class T>
struct GramStage {
  static constexpr int VE = 16 / (int)sizeof(T);           // elements per 16-byte load
  static constexpr int PER = kSlab * 64 / (256 * VE);       // loads per thread per panel
  static constexpr int LD = 64 + VE;                        // padded LDS row
};

template <class T>
__device__ inline void gram_load(const T* __restrict__ X, int64_t ldx, int ncol, int col0,
                                 int64_t k, int64_t ke, bool vec, T (&reg)[GramStage<T>::PER][GramStage<T>::VE]) {
  using S = GramStage<T>;
#pragma unroll
  for (int u = 0; u < S::PER; ++u) {
    const int e = (u * 256 + (int)threadIdx.x) * S::VE;  // element in the 32 x 64 panel
    const int r = e >> 6, c = e & 63;
    const int64_t row = k + r;
    const int col = col0 + c;
    if (vec && row < ke && col + S::VE <= ncol) {
      typedef T vec_t __attribute__((ext_vector_type(GramStage<T>::VE)));
      const vec_t v = *reinterpret_cast<const vec_t*>(X + row * ldx + col);
#pragma unroll
      for (int t = 0; t < S::VE; ++t) reg[u][t] = v[t];
    } else {
#pragma unroll
      for (int t = 0; t < S::VE; ++t)
        reg[u][t] = (row < ke && col + t < ncol) ? X[row * ldx + col + t] : (T)0;
    }
  }
}

template <class T>
__device__ inline void gram_store(T* __restrict__ sm, const T (&reg)[GramStage<T>::PER][GramStage<T>::VE]) {
  using S = GramStage<T>;
#pragma unroll
  for (int u = 0; u < S::PER; ++u) {
    const int e = (u * 256 + (int)threadIdx.x) * S::VE;
    const int r = e >> 6, c = e & 63;
#pragma unroll
    for (int t = 0; t < S::VE; ++t) sm[r * S::LD + c + t] = reg[u][t];
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_gram(int64_t n, const T* __restrict__ A, int64_t lda,
                                              int p, const T* __restrict__ B, int64_t ldb, int q,
                                              int sym, int vec, int64_t rows_per_split,
                                              double* __restrict__ part) {
  using M = Mfma<T>;
  using S = GramStage<T>;
  __shared__ T sa[kSlab * S::LD], sb[kSlab * S::LD];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wy = wave >> 1, wx = wave & 1;
  const int tiles_q = (q + 63) / 64;
  int ty, tx;
  if (sym) {
    int t = blockIdx.x;
    ty = 0;
    while (t >= tiles_q - ty) {
      t -= tiles_q - ty;
      ++ty;
    }
    tx = ty + t;
  } else {
    ty = blockIdx.x / tiles_q;
    tx = blockIdx.x % tiles_q;
  }
  const bool same = sym && ty == tx;  // one panel serves both operands
  const T* sbp = same ? sa : sb;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t kb = (int64_t)blockIdx.y * rows_per_split;
  const int64_t ke = min(n, kb + rows_per_split);
  typename M::acc acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = typename M::acc{0, 0, 0, 0};
  T ra[S::PER][S::VE], rb[S::PER][S::VE];
  if (kb < ke) {
    gram_load<T>(A, lda, p, ty * 64, kb, ke, vec != 0, ra);
    if (!same) gram_load<T>(B, ldb, q, tx * 64, kb, ke, vec != 0, rb);
  }
  for (int64_t k = kb; k < ke; k += kSlab) {
    __syncthreads();  // the previous slab's MFMAs are done with the LDS panels
    gram_store<T>(sa, ra);
    if (!same) gram_store<T>(sb, rb);
    __syncthreads();
    if (k + kSlab < ke) {
      gram_load<T>(A, lda, p, ty * 64, k + kSlab, ke, vec != 0, ra);
      if (!same) gram_load<T>(B, ldb, q, tx * 64, k + kSlab, ke, vec != 0, rb);
    }
#pragma unroll
    for (int kk = 0; kk < kSlab; kk += 4) {
      T a[2], b[2];
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        a[v] = sa[(kk + lk) * S::LD + wy * 32 + 16 * v + li];
        b[v] = sbp[(kk + lk) * S::LD + wx * 32 + 16 * v + li];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = M::op(a[i], b[j], acc[i][j]);
    }
  }
  const int c0 = ty * 64 + wy * 32, d0 = tx * 64 + wx * 32;
  double* out = part + (int64_t)blockIdx.y * p * q;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = c0 + 16 * i + M::row(lk, v);
        const int c = d0 + 16 * j + li;
        if (r < p && c < q) out[(int64_t)r * q + c] = (double)acc[i][j][v];
      }
}

// One wavefront per output element: lane l sums splits l, l+64, ... in order,
// then a fixed butterfly folds the 64 lane sums.
// sym: elements of tiles below the diagonal are read from their mirror.
__global__ __launch_bounds__(256) void k_gram_fold(const double* __restrict__ part, int splits,
                                                   int p, int q, int sym, double* __restrict__ C,
                                                   int64_t ldc) {
  const int lane = threadIdx.x & 63;
  const int64_t idx = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (idx >= (int64_t)p * q) return;
  const int r = (int)(idx / q), c = (int)(idx % q);
  const int64_t src = (sym && (r >> 6) > (c >> 6)) ? (int64_t)c * q + r : idx;
  double s = 0.0;
  for (int sp = lane; sp < splits; sp += 64) s += part[(int64_t)sp * p * q + src];
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) C[(idx / q) * ldc + idx % q] = s;
}

// Y[r, j] = sum_k A[r, k] C[k, j] + beta Y[r, j].  Tile: 64 rows x 64 columns
// per workgroup, 32-deep K slices in LDS; each thread owns 4 x 4 outputs.
template <class T>
__global__ __launch_bounds__(256) void k_combine(int64_t n, const T* __restrict__ A, int64_t lda,
                                                 int p, const double* __restrict__ Cm,
                                                 int64_t ldc, T* __restrict__ Y, int64_t ldy,
                                                 int q, double beta) {
  __shared__ T As[32][64 + 1];  // [k][row]
  __shared__ T Cs[32][64];      // [k][col]
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 64;
  const int tr = (tid >> 4) * 4, tc = (tid & 15) * 4;
  T acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (T)0;
  for (int k0 = 0; k0 < p; k0 += 32) {
    for (int e = tid; e < 32 * 64; e += 256) {
      const int rr = e >> 5, kk = e & 31;  // coalesced along k within a row
      const int64_t row = r0 + rr;
      const int col = k0 + kk;
      As[kk][rr] = (row < n && col < p) ? A[row * lda + col] : (T)0;
      const int ck = e >> 6, cc = e & 63;
      Cs[ck][cc] = (k0 + ck < p && c0 + cc < q) ? (T)Cm[(int64_t)(k0 + ck) * ldc + c0 + cc] : (T)0;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < 32; ++kk) {
      T av[4], cv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[kk][tr + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) cv[j] = Cs[kk][tc + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += av[i] * cv[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = r0 + tr + i;
    if (row >= n) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = c0 + tc + j;
      if (col >= q) continue;
      T* y = Y + row * ldy + col;
      *y = (beta == 0.0) ? acc[i][j] : (T)(acc[i][j] + (T)beta * *y);
    }
  }
}

template <class S, class D>
__global__ __launch_bounds__(256) void k_convert(int64_t n, int b, const S* __restrict__ X,
                                                 int64_t ldx, D* __restrict__ Y, int64_t ldy) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= n * b) return;
  const int64_t r = idx / b;
  const int c = (int)(idx % b);
  Y[r * ldy + c] = (D)X[r * ldx + c];
}

// Diagonal preconditioner of the extreme-eigenvalue iteration (sign*H):
// W[r,c] = R[r,c] / max(|sign*E_r - mu_c|, floor), with E the diagonal of H and
// mu the current Ritz values.
__global__ __launch_bounds__(256) void k_diag_precond(int64_t n, int b, const double* __restrict__ R,
                                                      int64_t ldr, const double* __restrict__ E,
                                                      double sign, const double* __restrict__ mu,
                                                      double floor, double* __restrict__ W,
                                                      int64_t ldw) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= n * b) return;
  const int64_t r = idx / b;
  const int c = (int)(idx % b);
  const double d = fmax(fabs(sign * E[r] - mu[c]), floor);
  W[r * ldw + c] = R[r * ldr + c] / d;
}

// splitmix64 (Steele, Lea, Flood 2014) of a counter, then Box-Muller.
__device__ inline uint64_t splitmix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

template <class T>
__global__ __launch_bounds__(256) void k_randn(int64_t n, int b, uint64_t seed, T* __restrict__ X,
                                               int64_t ldx) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= n * b) return;
  const uint64_t h1 = splitmix64(seed ^ splitmix64(2 * (uint64_t)idx));
  const uint64_t h2 = splitmix64(seed ^ splitmix64(2 * (uint64_t)idx + 1));
  const double u1 = ((h1 >> 11) + 1) * (1.0 / 9007199254740993.0);  // (0, 1]
  const double u2 = (h2 >> 11) * (1.0 / 9007199254740992.0);
  X[(idx / b) * ldx + idx % b] = (T)(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
}

inline unsigned g1(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

GramPlan gram_plan(int64_t n, int p, int q, bool same_operand) {
  GramPlan g;
  // A^T A: only the upper tiles (the Rayleigh-Ritz and Cholesky-QR Grams)
  g.sym = (same_operand && p == q) ? 1 : 0;
  const int tq = (q + 63) / 64;
  g.tiles = g.sym ? tq * (tq + 1) / 2 : ((p + 63) / 64) * tq;
  if (n == 0) {  // one split of zero rows: the kernel writes zero partials
    g.splits = 1;
    g.rows = kSlab;
  } else {
    int64_t splits = std::max<int64_t>(1, 1024 / g.tiles);
    splits = std::min<int64_t>(splits, std::max<int64_t>(1, (n + 255) / 256));
    int64_t rows = (n + splits - 1) / splits;
    rows = ((rows + kSlab - 1) / kSlab) * kSlab;
    g.rows = rows;
    g.splits = std::max<int64_t>(1, (n + rows - 1) / rows);
  }
  g.part_bytes = (size_t)g.splits * p * q * sizeof(double);
  return g;
}

template <class T>
void launch_gram_part(const GramPlan& g, int64_t n, const T* A, int64_t lda, int p, const T* B,
                      int64_t ldb, int q, double* C, int64_t ldc, double* part, hipStream_t s) {
  if (p == 0 || q == 0) return;
  PhaseTick tick(PhaseClock::GRAM, s);
  const uintptr_t align = reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B) |
                          (uintptr_t)(lda * (int64_t)sizeof(T)) |
                          (uintptr_t)(ldb * (int64_t)sizeof(T));
  const int vec = (align % 16) == 0;
  hipLaunchKernelGGL(k_gram<T>, dim3(g.tiles, (unsigned)g.splits), dim3(256), 0, s, n, A, lda, p,
                     B, ldb, q, g.sym, vec, g.rows, part);
  MBL_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_gram_fold, dim3((unsigned)(((int64_t)p * q + 3) / 4)), dim3(256), 0, s,
                     part, (int)g.splits, p, q, g.sym, C, ldc);
  MBL_CHECK_LAUNCH();
}

template <class T>
void launch_gram(int64_t n, const T* A, int64_t lda, int p, const T* B, int64_t ldb, int q,
                 double* C, int64_t ldc, hipStream_t s) {
  if (p == 0 || q == 0) return;
  const GramPlan g = gram_plan(n, p, q, A == B && lda == ldb);
  DevBuf part(g.part_bytes, s);
  launch_gram_part<T>(g, n, A, lda, p, B, ldb, q, C, ldc, part.as<double>(), s);
}

// ---- Gram partials in a fixed device array -------------------------------
// For callers that cannot allocate device memory (graph capture, tight
// loops): the per-split partial sums live in this file-scope array instead
// of a DevBuf.  Every k_gram launch writes each partial the fold reads, so
// nothing needs clearing between calls.  One copy per device; host code uses
// only the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[kGramScratchBytes / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};
}  // namespace

double* gram_scratch() {
  int dev = 0;
  MBL_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(MBL_EDEVICE, "device ordinal out of range for the Gram scratch");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[dev] == nullptr) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
      fail(MBL_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = static_cast<double*>(ptr);
  }
  return g_scratch[dev];
}

template <class T>
void launch_combine(int64_t n, const T* A, int64_t lda, int p, const double* C, int64_t ldc, T* Y,
                    int64_t ldy, int q, double beta, hipStream_t s) {
  if (n == 0 || q == 0) return;
  hipLaunchKernelGGL(k_combine<T>, dim3((unsigned)((n + 63) / 64), (unsigned)((q + 63) / 64)),
                     dim3(256), 0, s, n, A, lda, p, C, ldc, Y, ldy, q, beta);
  MBL_CHECK_LAUNCH();
}

template <class S, class D>
void launch_convert(int64_t n, int b, const S* X, int64_t ldx, D* Y, int64_t ldy, hipStream_t s) {
  if (n * b == 0) return;
  hipLaunchKernelGGL((k_convert<S, D>), dim3(g1(n * b)), dim3(256), 0, s, n, b, X, ldx, Y, ldy);
  MBL_CHECK_LAUNCH();
}

void launch_diag_precond(int64_t n, int b, const double* R, int64_t ldr, const double* E,
                         double sign, const double* mu, double floor, double* W, int64_t ldw,
                         hipStream_t s) {
  if (n * b == 0) return;
  hipLaunchKernelGGL(k_diag_precond, dim3(g1(n * b)), dim3(256), 0, s, n, b, R, ldr, E, sign, mu,
                     floor, W, ldw);
  MBL_CHECK_LAUNCH();
}

template <class T>
void launch_randn(int64_t n, int b, uint64_t seed, T* X, int64_t ldx, hipStream_t s) {
  if (n * b == 0) return;
  hipLaunchKernelGGL(k_randn<T>, dim3(g1(n * b)), dim3(256), 0, s, n, b, seed, X, ldx);
  MBL_CHECK_LAUNCH();
}

template void launch_gram<double>(int64_t, const double*, int64_t, int, const double*, int64_t,
                                  int, double*, int64_t, hipStream_t);
template void launch_gram<float>(int64_t, const float*, int64_t, int, const float*, int64_t, int,
                                 double*, int64_t, hipStream_t);
template void launch_gram_part<double>(const GramPlan&, int64_t, const double*, int64_t, int,
                                       const double*, int64_t, int, double*, int64_t, double*,
                                       hipStream_t);
template void launch_gram_part<float>(const GramPlan&, int64_t, const float*, int64_t, int,
                                      const float*, int64_t, int, double*, int64_t, double*,
                                      hipStream_t);
template void launch_combine<double>(int64_t, const double*, int64_t, int, const double*, int64_t,
                                     double*, int64_t, int, double, hipStream_t);
template void launch_combine<float>(int64_t, const float*, int64_t, int, const double*, int64_t,
                                    float*, int64_t, int, double, hipStream_t);
template void launch_convert<double, float>(int64_t, int, const double*, int64_t, float*, int64_t,
                                            hipStream_t);
template void launch_convert<float, double>(int64_t, int, const float*, int64_t, double*, int64_t,
                                            hipStream_t);
template void launch_convert<double, double>(int64_t, int, const double*, int64_t, double*,
                                             int64_t, hipStream_t);
template void launch_convert<float, float>(int64_t, int, const float*, int64_t, float*, int64_t,
                                           hipStream_t);
template void launch_randn<double>(int64_t, int, uint64_t, double*, int64_t, hipStream_t);
template void launch_randn<float>(int64_t, int, uint64_t, float*, int64_t, hipStream_t);

}  // namespace mbl
