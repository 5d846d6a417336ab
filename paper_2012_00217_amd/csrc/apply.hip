// Matrix-free block apply Y = (H - sigma I) X (paper Sec. 3.2 and 4.1) and the
// Jacobi-preconditioned CG on the spectral fold (H - sigma I)^2 built from it.
//
// Gather form (H is symmetric, so no atomics):
//   Y[r,:] = (E(s_r) - sigma) X[r,:] + (J/2) sum_{bonds i active in s_r} X[r +- C(i,t), :]
// with t = number of up spins below site i (see sector.hip for the identity).
//
// Layout: X, Y are row-major, n x b with leading dimension ld.  The columns
// are processed in chunks; within a chunk every lane owns NV vectors of VE
// contiguous elements (16 bytes when aligned), and G = 2^log2G lanes cover one
// row, so a wavefront covers 64/G consecutive rows.  Consecutive rows share
// their high bits, hence mostly the same active high bonds, which keeps the
// bond loop coherent across the wavefront.  Every gather of one bond reads
// G*NV*VE contiguous elements per row: whole 128-byte lines for wide chunks.
//
// Work distribution: row tiles of 4 waves x 64/G rows; the grid is a multiple
// of 8 and workgroup k runs on XCD k % 8, so each XCD walks runs of
// consecutive tiles and the low-bond neighbours (offsets C(i,t) small) of its
// rows stay in its own L2.  The run length (tiles per XCD group), workgroups
// per XCD, row-chunk and lane widths form the launch schedule, taken from a
// table the package's autotuner measured (apply_schedules.inc).
//
// Column reductions (the CG dot products) are accumulated in FP64 per lane,
// reduced across the wavefront with a fixed butterfly, across the 4 waves in
// LDS, written as one partial per workgroup ([column][workgroup], so the fold
// reads contiguously) and folded by a separate kernel in workgroup order, so
// every dot product is bitwise reproducible.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <exception>
#include <map>
#include <memory>
#include <mutex>

#include "common.h"

namespace mbl {
namespace {

template <class T, int VE>
struct alignas(sizeof(T) * VE) Pack {
  T v[VE];
};

#ifndef MBL_APPLY_NT_STORE
#define MBL_APPLY_NT_STORE 1
#endif

// Streaming store of one vector: outputs are not re-read by the same kernel,
// so they should not displace gathered rows of X from the L2.
template <class T, int VE>
__device__ inline void store_stream(T* p, const Pack<T, VE>& v) {
#if MBL_APPLY_NT_STORE
  if constexpr (VE == 1) {
    __builtin_nontemporal_store(v.v[0], p);
  } else {
    typedef T vec_t __attribute__((ext_vector_type(VE)));
    vec_t x;
#pragma unroll
    for (int e = 0; e < VE; ++e) x[e] = v.v[e];
    __builtin_nontemporal_store(x, reinterpret_cast<vec_t*>(p));
  }
#else
  *reinterpret_cast<Pack<T, VE>*>(p) = v;
#endif
}

// Cache hints of the CG vectors.  Measured on the MI355X (block PCG, tuned
// schedules): storing T with ordinary stores, or loading p, x, r with
// non-temporal loads, changes a CG step by -3.6% to +24% depending on the
// shape (the loads slow L = 18 down, where the whole working set stays in the
// caches), so both hints stay at the plain defaults below.
#ifndef MBL_CG_T_NT_STORE
#define MBL_CG_T_NT_STORE 1
#endif
#ifndef MBL_CG_NT_LOAD
#define MBL_CG_NT_LOAD 0
#endif

// Store of the CG intermediate T = (H - sigma) p, which the next kernel gathers.
template <class T, int VE>
__device__ inline void store_cg_t(T* p, const Pack<T, VE>& v) {
#if MBL_CG_T_NT_STORE
  store_stream<T, VE>(p, v);
#else
  *reinterpret_cast<Pack<T, VE>*>(p) = v;
#endif
}

// Load of a CG vector row that this kernel reads exactly once.
template <class T, int VE>
__device__ inline Pack<T, VE> load_once(const T* p) {
#if MBL_CG_NT_LOAD
  Pack<T, VE> r;
  if constexpr (VE == 1) {
    r.v[0] = __builtin_nontemporal_load(p);
  } else {
    typedef T vec_t __attribute__((ext_vector_type(VE)));
    const vec_t x = __builtin_nontemporal_load(reinterpret_cast<const vec_t*>(p));
#pragma unroll
    for (int e = 0; e < VE; ++e) r.v[e] = x[e];
  }
  return r;
#else
  return *reinterpret_cast<const Pack<T, VE>*>(p);
#endif
}

// Tile schedule.  Tiles are dealt to the 8 XCDs in groups: group g covers
// tiles [g*8*grp, (g+1)*8*grp) and XCD x takes the grp consecutive tiles
// starting at g*8*grp + x*grp.  grp = ceil(ntiles/8) gives each XCD one
// contiguous eighth of the rows; grp = 1 interleaves single tiles; values in
// between keep a compact sweep front (good for the shared MALL) while each
// XCD still sees runs of consecutive rows (good for its own L2).  Workgroup k
// runs on XCD k % 8; the workgroups of one XCD walk its tiles in order.
struct TileSched {
  int64_t ntiles;
  int grp;
};

__device__ inline int64_t sched_tile(const TileSched& t, int64_t u, int x, bool* done) {
  const int64_t g = u / t.grp;
  const int64_t base = g * 8 * t.grp;
  *done = base >= t.ntiles;
  return base + (int64_t)x * t.grp + (u - g * t.grp);
}

enum { EPI_PLAIN = 0, EPI_NORM2 = 1, EPI_PCG = 2 };

template <class T>
struct ApplyArgs {
  const uint32_t* states;
  const double* diag;
  const uint32_t* pascal;
  const T* X;
  int64_t ldx;
  T* Y;
  int64_t ldy;
  // EPI_PCG: the apply result is q = A p; x += alpha p, r -= alpha q.
  T* x;
  int64_t ldxv;
  T* r;
  int64_t ldr;
  const T* p;
  int64_t ldp;
  const T* jac;
  const PcgCoef* coef;
  double* part;
  int64_t n;
  double sigma, halfJ;
  int L;
  int col0, w, log2G;
  TileSched ts;
};

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;


template <class T, int VE, int NV>
__device__ inline void block_reduce_store(double (&red)[NV * VE], int log2G, int w,
                                          double* __restrict__ part, int bid, int nwg) {
  extern __shared__ double sred[];  // [kWaves][w]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int G = 1 << log2G;
#pragma unroll
  for (int k = 0; k < NV * VE; ++k)
    for (int off = G; off < 64; off <<= 1) red[k] += __shfl_xor(red[k], off);
  if (lane < G) {
#pragma unroll
    for (int q = 0; q < NV; ++q)
#pragma unroll
      for (int e = 0; e < VE; ++e) sred[wave * w + (q * G + lane) * VE + e] = red[q * VE + e];
  }
  __syncthreads();
  for (int c = threadIdx.x; c < w; c += kThreads) {
    double s = sred[c];
#pragma unroll
    for (int wv = 1; wv < kWaves; ++wv) s += sred[wv * w + c];
    part[(int64_t)c * nwg + bid] = s;  // [column][workgroup]
  }
}

// MBL_APPLY_ALPHA_LDS=1 (default): the fused CG update reads its step lengths
// from LDS instead of holding them in registers, which brings the FP32
// 128-column CG kernel from 177 to 165 registers (3 waves per SIMD instead of
// 2; about 2% faster per CG step at L = 22 and 24).
#ifndef MBL_APPLY_ALPHA_LDS
#define MBL_APPLY_ALPHA_LDS 1
#endif

#ifndef MBL_APPLY_BB_BYTES
#define MBL_APPLY_BB_BYTES 256
#endif

constexpr int kNoFlip = -2147483647 - 1;  // offset-table entry of an inactive bond

// One wavefront owns RW = 64/G consecutive rows per tile.  Phase A fills the
// wave's LDS table off[r][i] (r < RW, i < 32) with the row offset of the flip
// target of bond i in row r, or kNoFlip: the RW*32 entries are spread over all
// 64 lanes, so each flip target is computed exactly once.  Phase B: the G
// lanes of a row read four offsets at a time (one LDS load) and gather the
// target rows' column chunks.
template <class T, int VE, int NV, int EPI>
__device__ __forceinline__ void apply_body(const ApplyArgs<T>& a, const int bid, const int nwg) {
  using P = Pack<T, VE>;
  constexpr int BB0 = MBL_APPLY_BB_BYTES / (NV * VE * (int)sizeof(T));
  constexpr int BB = BB0 <= 1 ? 1 : (BB0 >= 4 ? 4 : 2);  // bonds per batch of loads
  __shared__ uint32_t C[kPascal * kPascal];
  extern __shared__ double sdyn[];  // [kWaves][w] doubles for reductions, then offset tables
  for (int i = threadIdx.x; i < kPascal * kPascal; i += kThreads) C[i] = a.pascal[i];

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int G = 1 << a.log2G;
  const int RW = 64 >> a.log2G;
  const int rsub = lane >> a.log2G;
  const int cl = lane & (G - 1);
  const int nb = a.L - 1;
  const uint32_t bondmask = nb > 0 ? ((1u << nb) - 1u) : 0u;
  const int cbase = a.col0 + cl * VE;  // first column of unit 0 of this lane
  const int red_doubles = (EPI == EPI_PLAIN) ? 0 : kWaves * a.w;
  int* offtab = reinterpret_cast<int*>(sdyn + red_doubles) + wave * (RW * 32);
  __syncthreads();

  double red[NV * VE];
#pragma unroll
  for (int k = 0; k < NV * VE; ++k) red[k] = 0.0;
#if MBL_APPLY_ALPHA_LDS
  // the CG step lengths of the chunk's columns in LDS (after the offset
  // tables), read per row instead of held in registers
  T* salpha = reinterpret_cast<T*>(reinterpret_cast<int*>(sdyn + red_doubles) + kWaves * RW * 32);
  if constexpr (EPI == EPI_PCG) {
    for (int c = threadIdx.x; c < a.w; c += kThreads) salpha[c] = (T)a.coef[a.col0 + c].alpha;
    __syncthreads();
  }
#else
  T alpha[NV * VE];
  if constexpr (EPI == EPI_PCG) {
#pragma unroll
    for (int q = 0; q < NV; ++q)
#pragma unroll
      for (int e = 0; e < VE; ++e) alpha[q * VE + e] = (T)a.coef[cbase + q * G * VE + e].alpha;
  }
#endif
  const T hj = (T)a.halfJ;

  const int xcd = bid & 7;
  const int nslots = nwg >> 3;
  for (int64_t u = bid >> 3;; u += nslots) {
    bool done;
    const int64_t tile = sched_tile(a.ts, u, xcd, &done);
    if (done) break;
    if (tile >= a.ts.ntiles) continue;
    const int64_t row0 = tile * (kWaves * RW) + wave * RW;  // first row of this wave

    // Phase A: flip targets of the wave's RW rows, 32 bond slots per row.
    for (int it = lane; it < RW * 32; it += 64) {
      const int r = it >> 5, i = it & 31;
      const int64_t rr = row0 + r;
      int o = kNoFlip;
      if (rr < a.n && i < nb) {
        const uint32_t sr = a.states[rr];
        if (((sr ^ (sr >> 1)) >> i) & 1u) {
          const int c = (int)C[i * kPascal + __popc(sr & ((1u << i) - 1u))];
          const int d = ((sr >> i) & 1u) ? c : -c;
          // the flip identity keeps the target in [0, n); the guard makes a
          // corrupted state table drop a term instead of reading out of bounds
          if (rr + d >= 0 && rr + d < a.n) o = d;
        }
      }
      offtab[it] = o;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // Phase B: gather for this lane's row.
    const int64_t row = row0 + rsub;
    if (row < a.n) {
      const T* xrow = a.X + row * a.ldx + cbase;
      P own[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) own[q] = *reinterpret_cast<const P*>(xrow + q * G * VE);
      T nbs[NV * VE];
#pragma unroll
      for (int k = 0; k < NV * VE; ++k) nbs[k] = (T)0;
      const int* myoff = offtab + rsub * 32;
      for (int i0 = 0; i0 < nb; i0 += BB) {
        int o[BB];
#pragma unroll
        for (int v = 0; v < BB; ++v) o[v] = myoff[i0 + v];
        P v[BB][NV];
#pragma unroll
        for (int b2 = 0; b2 < BB; ++b2) {
          if (o[b2] != kNoFlip) {
            const T* xp = xrow + (int64_t)o[b2] * a.ldx;
#pragma unroll
            for (int q = 0; q < NV; ++q) v[b2][q] = *reinterpret_cast<const P*>(xp + q * G * VE);
          } else {
#pragma unroll
            for (int q = 0; q < NV; ++q)
#pragma unroll
              for (int e = 0; e < VE; ++e) v[b2][q].v[e] = (T)0;
          }
        }
#pragma unroll
        for (int b2 = 0; b2 < BB; ++b2)
#pragma unroll
          for (int q = 0; q < NV; ++q)
#pragma unroll
            for (int e = 0; e < VE; ++e) nbs[q * VE + e] += v[b2][q].v[e];
      }
      const T ed = (T)(a.diag[row] - a.sigma);
      T acc[NV * VE];
#pragma unroll
      for (int q = 0; q < NV; ++q)
#pragma unroll
        for (int e = 0; e < VE; ++e) acc[q * VE + e] = ed * own[q].v[e] + hj * nbs[q * VE + e];

      if constexpr (EPI == EPI_PLAIN || EPI == EPI_NORM2) {
        T* yr = a.Y + row * a.ldy + cbase;
#pragma unroll
        for (int q = 0; q < NV; ++q) {
          P o2;
#pragma unroll
          for (int e = 0; e < VE; ++e) o2.v[e] = acc[q * VE + e];
          if constexpr (EPI == EPI_NORM2)
            store_cg_t<T, VE>(yr + q * G * VE, o2);
          else
            store_stream<T, VE>(yr + q * G * VE, o2);
        }
        if constexpr (EPI == EPI_NORM2) {
#pragma unroll
          for (int k = 0; k < NV * VE; ++k) red[k] += (double)acc[k] * (double)acc[k];
        }
      } else {  // EPI_PCG
        const T* pr = a.p + row * a.ldp + cbase;
        T* xr = a.x + row * a.ldxv + cbase;
        T* rr = a.r + row * a.ldr + cbase;
        const T dinv = (T)1 / a.jac[row];
#pragma unroll
        for (int q = 0; q < NV; ++q) {
          P pv = load_once<T, VE>(pr + q * G * VE);
          P xv = load_once<T, VE>(xr + q * G * VE);
          P rv = load_once<T, VE>(rr + q * G * VE);
#if MBL_APPLY_ALPHA_LDS
          const P av = *reinterpret_cast<const P*>(salpha + (cbase - a.col0) + q * G * VE);
#endif
#pragma unroll
          for (int e = 0; e < VE; ++e) {
#if MBL_APPLY_ALPHA_LDS
            const T al = av.v[e];
#else
            const T al = alpha[q * VE + e];
#endif
            xv.v[e] = xv.v[e] + al * pv.v[e];
            rv.v[e] = rv.v[e] - al * acc[q * VE + e];
            red[q * VE + e] += (double)rv.v[e] * (double)(rv.v[e] * dinv);
          }
          store_stream<T, VE>(xr + q * G * VE, xv);
          store_stream<T, VE>(rr + q * G * VE, rv);
        }
      }
    }
    // the next tile's phase A overwrites this wave's table
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  if constexpr (EPI != EPI_PLAIN) block_reduce_store<T, VE, NV>(red, a.log2G, a.w, a.part, bid, nwg);
}

// MBL_APPLY_WAVES > 0 asks the compiler for at least that many waves per SIMD
// (a register cap) on the apply kernels; 0 leaves the choice to it.
#ifndef MBL_APPLY_WAVES
#define MBL_APPLY_WAVES 0
#endif
#if MBL_APPLY_WAVES > 0
#define MBL_APPLY_OCC __attribute__((amdgpu_waves_per_eu(MBL_APPLY_WAVES, 8)))
#else
#define MBL_APPLY_OCC
#endif

template <class T, int VE, int NV, int EPI>
__global__ __launch_bounds__(kThreads) MBL_APPLY_OCC void k_apply(ApplyArgs<T> a) {
  apply_body<T, VE, NV, EPI>(a, blockIdx.x, gridDim.x);
}

// Several problems in one launch (the fused CG of a batch): problem j owns
// workgroups [wg0[j], wg0[j+1]); every wg0[j] is a multiple of 8, so each
// problem's workgroups keep their XCDs, tiles and partial-sum slots of a launch
// of their own, and the results are the same bits.
constexpr int kMaxFuse = 8;

template <class T>
struct MultiApply {
  int np;
  int wg0[kMaxFuse + 1];
  ApplyArgs<T> a[kMaxFuse];
};

template <class T, int VE, int NV, int EPI>
__global__ __launch_bounds__(kThreads) MBL_APPLY_OCC void k_apply_multi(MultiApply<T> m) {
  int j = 0;
  while (j + 1 < m.np && (int)blockIdx.x >= m.wg0[j + 1]) ++j;
  apply_body<T, VE, NV, EPI>(m.a[j], (int)blockIdx.x - m.wg0[j], m.wg0[j + 1] - m.wg0[j]);
}

// PCG element-wise kernels with the same lane layout as k_apply.
enum { ELT_INIT = 0, ELT_PUPD = 1 };

template <class T>
struct EltArgs {
  const T* R;  // INIT: right-hand side
  int64_t ldR;
  T* x;
  int64_t ldxv;
  T* r;
  int64_t ldr;
  T* p;
  int64_t ldp;
  const T* jac;
  const PcgCoef* coef;
  double* part;
  int64_t n;
  int col0, w, log2G;
  TileSched ts;
};

template <class T, int VE, int NV, int MODE>
__device__ __forceinline__ void elt_body(const EltArgs<T>& a, const int bid, const int nwg) {
  using P = Pack<T, VE>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int G = 1 << a.log2G;
  const int RW = 64 >> a.log2G;
  const int rsub = lane >> a.log2G;
  const int cl = lane & (G - 1);
  const int cbase = a.col0 + cl * VE;
  double red[NV * VE];
#pragma unroll
  for (int k = 0; k < NV * VE; ++k) red[k] = 0.0;
  T beta[NV * VE];
  bool live[NV * VE];
  if constexpr (MODE == ELT_PUPD) {
#pragma unroll
    for (int q = 0; q < NV; ++q)
#pragma unroll
      for (int e = 0; e < VE; ++e) {
        const PcgCoef& c = a.coef[cbase + q * G * VE + e];
        beta[q * VE + e] = (T)c.beta;
        live[q * VE + e] = c.live != 0;
      }
  }
  const int xcd = bid & 7;
  const int nslots = nwg >> 3;
  for (int64_t u = bid >> 3;; u += nslots) {
    bool done;
    const int64_t tile = sched_tile(a.ts, u, xcd, &done);
    if (done) break;
    if (tile >= a.ts.ntiles) continue;
    const int64_t row = tile * (kWaves * RW) + wave * RW + rsub;
    if (row >= a.n) continue;
    const T dinv = (T)1 / a.jac[row];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int64_t off = cbase + q * G * VE;
      if constexpr (MODE == ELT_INIT) {
        P rv = *reinterpret_cast<const P*>(a.R + row * a.ldR + off);
        P xv, pv;
#pragma unroll
        for (int e = 0; e < VE; ++e) {
          xv.v[e] = (T)0;
          pv.v[e] = rv.v[e] * dinv;
          red[q * VE + e] += (double)rv.v[e] * (double)pv.v[e];
        }
        if (a.r != a.R) *reinterpret_cast<P*>(a.r + row * a.ldr + off) = rv;
        *reinterpret_cast<P*>(a.x + row * a.ldxv + off) = xv;
        *reinterpret_cast<P*>(a.p + row * a.ldp + off) = pv;
      } else {
        P rv = load_once<T, VE>(a.r + row * a.ldr + off);
        P pv = load_once<T, VE>(a.p + row * a.ldp + off);
#pragma unroll
        for (int e = 0; e < VE; ++e)
          if (live[q * VE + e]) pv.v[e] = rv.v[e] * dinv + beta[q * VE + e] * pv.v[e];
        *reinterpret_cast<P*>(a.p + row * a.ldp + off) = pv;
      }
    }
  }
  if constexpr (MODE == ELT_INIT) block_reduce_store<T, VE, NV>(red, a.log2G, a.w, a.part, bid, nwg);
}

template <class T, int VE, int NV, int MODE>
__global__ __launch_bounds__(kThreads) void k_pcg_elt(EltArgs<T> a) {
  elt_body<T, VE, NV, MODE>(a, blockIdx.x, gridDim.x);
}

template <class T>
struct MultiElt {
  int np;
  int wg0[kMaxFuse + 1];
  EltArgs<T> a[kMaxFuse];
};

template <class T, int VE, int NV, int MODE>
__global__ __launch_bounds__(kThreads) void k_pcg_elt_multi(MultiElt<T> m) {
  int j = 0;
  while (j + 1 < m.np && (int)blockIdx.x >= m.wg0[j + 1]) ++j;
  elt_body<T, VE, NV, MODE>(m.a[j], (int)blockIdx.x - m.wg0[j], m.wg0[j + 1] - m.wg0[j]);
}

// Fold the per-workgroup partials of one chunk (fixed order) and update the
// CG coefficients of its columns.  One workgroup per column: each thread sums
// a fixed strided subset, then the wavefronts (butterfly) and the workgroup
// (LDS, wave order) combine them.
enum { FIN_INIT = 0, FIN_ALPHA = 1, FIN_BETA = 2 };

template <int MODE>
__device__ __forceinline__ void fin_body(const double* __restrict__ part, int nwg, int col0,
                                         PcgCoef* __restrict__ coef, int c) {
  __shared__ double swave[kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double s = 0.0;
  const double* pc = part + (int64_t)c * nwg;
  for (int g = threadIdx.x; g < nwg; g += kThreads) s += pc[g];
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) swave[wave] = s;
  __syncthreads();
  if (threadIdx.x != 0) return;
  s = swave[0];
  for (int v = 1; v < kWaves; ++v) s += swave[v];
  PcgCoef& k = coef[col0 + c];
  if (MODE == FIN_INIT) {
    k.rho = s;
    k.live = s > 0.0;
    k.alpha = 0.0;
    k.beta = 0.0;
    k.pap = 0.0;
  } else if (MODE == FIN_ALPHA) {
    k.pap = s;
    k.live = k.live && (s > 0.0);
    k.alpha = k.live ? k.rho / s : 0.0;
  } else {
    k.live = k.live && (s > 0.0);
    k.beta = k.live ? s / k.rho : 0.0;
    if (k.live) k.rho = s;
  }
}

template <int MODE>
__global__ __launch_bounds__(kThreads) void k_pcg_finalize(const double* __restrict__ part,
                                                           int nwg, int w, int col0,
                                                           PcgCoef* __restrict__ coef) {
  if ((int)blockIdx.x >= w) return;  // uniform over the workgroup
  fin_body<MODE>(part, nwg, col0, coef, blockIdx.x);
}

// One workgroup per (problem, column): problem j owns workgroups
// [c0[j], c0[j+1]), one per column of its chunk.
struct MultiFin {
  int np;
  int c0[kMaxFuse + 1];
  const double* part[kMaxFuse];
  int nwg[kMaxFuse];
  int col0[kMaxFuse];
  PcgCoef* coef[kMaxFuse];
};

template <int MODE>
__global__ __launch_bounds__(kThreads) void k_pcg_finalize_multi(MultiFin m) {
  int j = 0;
  while (j + 1 < m.np && (int)blockIdx.x >= m.c0[j + 1]) ++j;
  fin_body<MODE>(m.part[j], m.nwg[j], m.col0[j], m.coef[j], (int)blockIdx.x - m.c0[j]);
}

struct Chunk {
  int col0, w, VE, NV, log2G;
};

int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v ? std::atoi(v) : dflt;
}

// Launch schedule of the apply and CG kernels: bytes of a row chunk, bytes
// per lane, tiles per XCD group (0 = one group per XCD) and workgroups per XCD.
struct Sched {
  int chunk_bytes, lane_bytes, grp, slots;
};

// Schedules measured best on the MI355X by the package's autotuner, keyed by
// chain length, sector dimension, bytes per row of the block and element size.
struct SchedEntry {
  int L;
  int64_t n;
  int row_bytes, elem;
  Sched s;
};
#include "apply_schedules.inc"

constexpr Sched kDefaultSched{512, 64, 0, 256};

// Table entry with the same element size and row width whose sector dimension
// is closest (within a factor 2.5) to n, else the default; each MBL_APPLY_*
// environment variable that is set overrides its field.
Sched sched_for(const Ham& H, int row_bytes, int elem) {
  Sched best = kDefaultSched;
  double dist = std::log(2.5);
  for (const SchedEntry& e : kSchedTable) {
    if (e.L == 0 || e.elem != elem || e.row_bytes != row_bytes) continue;
    const double d = std::fabs(std::log((double)e.n / (double)std::max<int64_t>(1, H.n)));
    if (d <= dist) {
      dist = d;
      best = e.s;
    }
  }
  best.chunk_bytes = env_int("MBL_APPLY_CHUNK_BYTES", best.chunk_bytes);
  best.lane_bytes = env_int("MBL_APPLY_LANE_BYTES", best.lane_bytes);
  best.grp = env_int("MBL_APPLY_XCD_GROUP", best.grp);
  best.slots = env_int("MBL_APPLY_SLOTS_PER_XCD", best.slots);
  return best;
}

// Split columns [0, b) into chunks of at most sc.chunk_bytes per row.
template <class T>
std::vector<Chunk> plan_chunks(int b, bool aligned16, const Sched& sc) {
  const int max_bytes = std::max(16, sc.chunk_bytes);
  std::vector<Chunk> out;
  const int VEv = aligned16 ? (int)(16 / sizeof(T)) : 1;
  int c = 0;
  while (c < b) {
    int VE = VEv;
    int units = (b - c) / VE;
    if (units == 0) {
      VE = 1;
      units = b - c;
    }
    const int lane_units = std::max(1, sc.lane_bytes / (int)(VE * sizeof(T)));
    int NV = 1;
    while (NV * 2 <= std::min(units, std::min(lane_units, VE > 1 ? 8 : 4))) NV *= 2;
    int G = std::min(64, units / NV);
    G = std::min(G, std::max(1, max_bytes / (int)(NV * VE * sizeof(T))));
    int log2G = 0;
    while ((2 << log2G) <= G) ++log2G;
    G = 1 << log2G;
    out.push_back({c, G * NV * VE, VE, NV, log2G});
    c += G * NV * VE;
  }
  return out;
}

bool al16(const void* p, int64_t ld, size_t es) {
  return (reinterpret_cast<uintptr_t>(p) % 16 == 0) && ((ld * (int64_t)es) % 16 == 0);
}

struct Grid {
  TileSched ts;
  unsigned nwg;
};

Grid make_grid(int64_t n, int log2G, const Sched& sc) {
  const int64_t rows_per_tile = kWaves * (64 >> log2G);
  Grid g;
  g.ts.ntiles = (n + rows_per_tile - 1) / rows_per_tile;
  const int64_t per_xcd = (g.ts.ntiles + 7) / 8;
  const int grp_knob = sc.grp;
  g.ts.grp = (int)std::max<int64_t>(1, grp_knob > 0 ? std::min<int64_t>(grp_knob, per_xcd) : per_xcd);
  const int64_t max_slots = std::min(256, std::max(1, sc.slots));
  const int64_t slots = std::min<int64_t>(per_xcd, max_slots);
  g.nwg = (unsigned)(8 * std::max<int64_t>(1, slots));
  return g;
}

constexpr int kMaxWg = 8 * 256;  // upper bound of Grid::nwg with the default knob

template <class T, int EPI>
void dispatch_apply(const Chunk& ch, const Grid& g, ApplyArgs<T> a, hipStream_t s) {
  a.col0 = ch.col0;
  a.w = ch.w;
  a.log2G = ch.log2G;
  a.ts = g.ts;
  const size_t shm = ((EPI == EPI_PLAIN) ? 0 : (size_t)kWaves * ch.w * sizeof(double)) +
                     (size_t)kWaves * (64 >> ch.log2G) * 32 * sizeof(int) +
                     ((MBL_APPLY_ALPHA_LDS && EPI == EPI_PCG) ? (size_t)ch.w * sizeof(T) : 0);
  constexpr int VV = 16 / sizeof(T);
#define MBL_APPLY_CASE(VE_, NV_)                                                             \
  if (ch.VE == VE_ && ch.NV == NV_) {                                                       \
    hipLaunchKernelGGL((k_apply<T, VE_, NV_, EPI>), dim3(g.nwg), dim3(kThreads), shm, s, a); \
    MBL_CHECK_LAUNCH();                                                                     \
    return;                                                                                 \
  }
  MBL_APPLY_CASE(VV, 8)
  MBL_APPLY_CASE(VV, 4)
  MBL_APPLY_CASE(VV, 2)
  MBL_APPLY_CASE(VV, 1)
  MBL_APPLY_CASE(1, 4)
  MBL_APPLY_CASE(1, 2)
  MBL_APPLY_CASE(1, 1)
#undef MBL_APPLY_CASE
  fail(MBL_EINTERNAL, "apply: no kernel for chunk shape");
}

template <class T, int MODE>
void dispatch_elt(const Chunk& ch, const Grid& g, EltArgs<T> a, hipStream_t s) {
  a.col0 = ch.col0;
  a.w = ch.w;
  a.log2G = ch.log2G;
  a.ts = g.ts;
  const size_t shm = (MODE == ELT_INIT) ? (size_t)kWaves * ch.w * sizeof(double) : 0;
  constexpr int VV = 16 / sizeof(T);
#define MBL_ELT_CASE(VE_, NV_)                                                                 \
  if (ch.VE == VE_ && ch.NV == NV_) {                                                         \
    hipLaunchKernelGGL((k_pcg_elt<T, VE_, NV_, MODE>), dim3(g.nwg), dim3(kThreads), shm, s, a); \
    MBL_CHECK_LAUNCH();                                                                       \
    return;                                                                                   \
  }
  MBL_ELT_CASE(VV, 8)
  MBL_ELT_CASE(VV, 4)
  MBL_ELT_CASE(VV, 2)
  MBL_ELT_CASE(VV, 1)
  MBL_ELT_CASE(1, 4)
  MBL_ELT_CASE(1, 2)
  MBL_ELT_CASE(1, 1)
#undef MBL_ELT_CASE
  fail(MBL_EINTERNAL, "pcg: no kernel for chunk shape");
}

template <int MODE>
void finalize(const Chunk& ch, const Grid& g, const double* part, PcgCoef* coef, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_finalize<MODE>, dim3(ch.w), dim3(kThreads), 0,
                     s, part, (int)g.nwg, ch.w, ch.col0, coef);
  MBL_CHECK_LAUNCH();
}

template <class T>
ApplyArgs<T> base_args(const Ham& H, double sigma) {
  ApplyArgs<T> a{};
  a.states = H.states.as<uint32_t>();
  a.diag = H.diag.as<double>();
  a.pascal = H.pascal.as<uint32_t>();
  a.n = H.n;
  a.sigma = sigma;
  a.halfJ = 0.5 * H.J;
  a.L = H.L;
  return a;
}

}  // namespace

template <class T>
void launch_apply(const Ham& H, double sigma, const T* X, int64_t ldx, T* Y, int64_t ldy, int w,
                  hipStream_t s) {
  if (H.n == 0 || w == 0) return;
  PhaseTick tick(PhaseClock::APPLY, s);
  if (split_apply<T>(H, sigma, X, ldx, Y, ldy, w, s)) return;
  const bool aligned = al16(X, ldx, sizeof(T)) && al16(Y, ldy, sizeof(T));
  ApplyArgs<T> a = base_args<T>(H, sigma);
  a.X = X;
  a.ldx = ldx;
  a.Y = Y;
  a.ldy = ldy;
  const Sched sc = sched_for(H, w * (int)sizeof(T), (int)sizeof(T));
  for (const Chunk& ch : plan_chunks<T>(w, aligned, sc))
    dispatch_apply<T, EPI_PLAIN>(ch, make_grid(H.n, ch.log2G, sc), a, s);
}

// Block Jacobi-PCG on A = (H - sigma)^2, x0 = 0, m steps, per column:
//   r = R, p = M^-1 r, rho = r.M^-1 r
//   repeat: T = (H-sigma) p ; alpha = rho / |T|^2          (p.A p = |T|^2)
//           q = (H-sigma) T ; x += alpha p ; r -= alpha q ; rho' = r.M^-1 r
//           beta = rho'/rho ; p = M^-1 r + beta p
// Every coefficient stays on the device; no host synchronisation inside.
void PcgTiming::init() {
  if (ready) return;
  for (auto& e : ev) MBL_HIP(hipEventCreate(&e));
  ready = true;
}

PcgTiming::~PcgTiming() {
  if (!ready) return;
  for (auto& e : ev) (void)hipEventDestroy(e);
}

// Columns of the block CG are independent, so the block can be solved one
// column chunk at a time; only the summation order of the dot products can
// change (the lane layout depends on the chunk width).  The chunk width is
// chosen so that the chunk's working set (r, p, T, x: 4 n w s bytes) fits a
// cache budget (MBL_PCG_CACHE_MB; off by default: measured slower at L = 20,
// where narrow chunks cost more per row than the cache saves).  When even a
// chunk of 64-byte rows does not fit, the whole block is one chunk.
template <class T>
int pcg_chunk_width(int64_t n, int b) {
  const char* env = std::getenv("MBL_PCG_CACHE_MB");
  const double budget = 1e6 * std::max(0.0, env ? std::atof(env) : 0.0);
  const int min_w = std::max(1, 64 / (int)sizeof(T));
  const double per_col = 4.0 * (double)n * sizeof(T) + 16.0 * n / std::max(1, b);
  int w = 1;
  while (w * 2 <= b && (double)(w * 2) * per_col <= budget) w *= 2;
  if (w < min_w || (double)w * per_col > budget) return b;
  return w;
}

// Replays `step` m - it times: from a hipGraph captured on a private
// non-blocking stream (forked from and joined back to s by events) when at
// least 8 steps remain, else launch by launch.  The legacy default stream
// cannot be captured, and a capture on a caller's blocking stream would forbid
// legacy-stream work in every other thread of the process meanwhile.
// With a stop check the replays are issued in chunks of kStopChunk, one chunk
// queued ahead of the one running, and no further chunk is issued once the
// check triggers.  Returns the number of steps run.
constexpr int kStopChunk = 32;

template <class F>
int replay_steps(F&& step, int it, int m, hipStream_t& s, const StopCheck* stop) {
  if (env_int("MBL_PCG_GRAPH", 1) != 0 && m - it >= 8) {
    hipStream_t own = nullptr;
    hipEvent_t fork = nullptr, join = nullptr, mark[2] = {nullptr, nullptr};
    MBL_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
    hipError_t err = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    if (err == hipSuccess) err = hipEventCreateWithFlags(&join, hipEventDisableTiming);
    for (int k = 0; k < 2 && err == hipSuccess; ++k)
      err = hipEventCreateWithFlags(&mark[k], hipEventDisableTiming);
    if (err == hipSuccess) err = hipEventRecord(fork, s);
    if (err == hipSuccess) err = hipStreamWaitEvent(own, fork, 0);
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (err == hipSuccess) err = hipStreamBeginCapture(own, hipStreamCaptureModeThreadLocal);
    if (err == hipSuccess) {
      const hipStream_t keep = s;
      s = own;  // step() launches on s
      try {
        step();
      } catch (...) {
        s = keep;
        hipGraph_t dropped = nullptr;
        (void)hipStreamEndCapture(own, &dropped);
        if (dropped) (void)hipGraphDestroy(dropped);
        (void)hipStreamSynchronize(own);
        (void)hipStreamDestroy(own);
        (void)hipEventDestroy(fork);
        (void)hipEventDestroy(join);
        for (hipEvent_t e : mark)
          if (e) (void)hipEventDestroy(e);
        throw;
      }
      s = keep;
      err = hipStreamEndCapture(own, &graph);
    }
    if (err == hipSuccess) err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    int chunk = 0;
    while (err == hipSuccess && it < m) {
      const int end = stop ? std::min(m, it + kStopChunk) : m;
      for (; err == hipSuccess && it < end; ++it) err = hipGraphLaunch(exec, own);
      if (!stop || err != hipSuccess || it >= m) continue;
      // wait for the chunk before this one, then decide whether to go on
      err = hipEventRecord(mark[chunk & 1], own);
      if (err == hipSuccess && chunk > 0) err = hipEventSynchronize(mark[(chunk - 1) & 1]);
      ++chunk;
      if (err == hipSuccess && stop->triggered()) break;
    }
    if (err == hipSuccess) err = hipEventRecord(join, own);
    if (err == hipSuccess) err = hipStreamWaitEvent(s, join, 0);
    // the graph and its stream are torn down only after the replays finished
    const hipError_t se = hipStreamSynchronize(own);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(own);
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    for (hipEvent_t e : mark)
      if (e) (void)hipEventDestroy(e);
    MBL_HIP(err);
    MBL_HIP(se);
    return it;
  }
  for (; it < m; ++it) {
    if (stop && it % kStopChunk == 0 && stop->triggered()) break;
    step();
  }
  return it;
}

// Block PCG of one column chunk through the split (two-pass) kernels:
//   init: r = R, x = 0, p = M^-1 r, rho = r.M^-1 r   (beta = 0)
//   step: [p = M^-1 r + beta p; T = (H - sigma) p; |T|^2] -> alpha
//         [q = (H - sigma) T; x += alpha p; r -= alpha q; r.M^-1 r] -> beta
// The p-update of each step is fused into the first apply of the next, which
// with beta = 0 after init reproduces p = M^-1 r.
template <class T>
void run_pcg_split(const Ham& H, double sigma, const T* jac, const T* Rc, int64_t ldr,
                   const SplitCg<T>& sg, int m, bool aligned, const Sched& sc, hipStream_t s,
                   PcgTiming* tm, const StopCheck* stop) {
  const int64_t n = H.n;
  const int w = sg.w;
  for (const Chunk& ch : plan_chunks<T>(w, aligned, sc)) {
    const Grid g = make_grid(n, ch.log2G, sc);
    EltArgs<T> e{};
    e.R = Rc;
    e.ldR = ldr;
    e.x = sg.x;
    e.ldxv = sg.ldx;
    e.r = sg.r;
    e.ldr = sg.ldr;
    e.p = sg.p;
    e.ldp = sg.ldp;
    e.jac = jac;
    e.coef = sg.coef;
    e.part = sg.part;
    e.n = n;
    dispatch_elt<T, ELT_INIT>(ch, g, e, s);
    finalize<FIN_INIT>(ch, g, sg.part, const_cast<PcgCoef*>(sg.coef), s);
  }
  auto fin = [&](int nwp, auto mode, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_finalize<decltype(mode)::value>, dim3(w), dim3(kThreads), 0, st,
                       sg.part, nwp, w, 0, const_cast<PcgCoef*>(sg.coef));
    MBL_CHECK_LAUNCH();
  };
  using FA = std::integral_constant<int, FIN_ALPHA>;
  using FB = std::integral_constant<int, FIN_BETA>;
  const int ntimed = tm ? std::min(m, PcgTiming::kSample) : 0;
  if (tm) tm->init();
  int it = 0;
  for (; it < ntimed; ++it) {
    MBL_HIP(hipEventRecord(tm->ev[4 * it + 0], s));
    int nwp = split_cg_apply<T>(H, sigma, 0, sg, s);
    MBL_HIP(hipEventRecord(tm->ev[4 * it + 1], s));
    fin(nwp, FA{}, s);
    MBL_HIP(hipEventRecord(tm->ev[4 * it + 2], s));
    nwp = split_cg_apply<T>(H, sigma, 1, sg, s);
    MBL_HIP(hipEventRecord(tm->ev[4 * it + 3], s));
    fin(nwp, FB{}, s);
  }
  auto step = [&]() {
    const int nwp1 = split_cg_apply<T>(H, sigma, 0, sg, s);
    fin(nwp1, FA{}, s);
    const int nwp2 = split_cg_apply<T>(H, sigma, 1, sg, s);
    fin(nwp2, FB{}, s);
  };
  const int run = replay_steps(step, it, m, s, stop);
  if (ntimed > 0) {
    MBL_HIP(hipStreamSynchronize(s));
    double sa = 0.0, sc = 0.0;
    for (int k = 0; k < ntimed; ++k) {
      float ta = 0.f, tc = 0.f;
      MBL_HIP(hipEventElapsedTime(&ta, tm->ev[4 * k + 0], tm->ev[4 * k + 1]));
      MBL_HIP(hipEventElapsedTime(&tc, tm->ev[4 * k + 2], tm->ev[4 * k + 3]));
      sa += ta;
      sc += tc;
    }
    // algorithmic bytes: apply1 (p-update fused) reads r, p and writes p, T;
    // apply2 reads T, p, x, r and writes x, r
    const double b1 = 4.0 * n * w * sizeof(T), b2 = 6.0 * n * w * sizeof(T);
    tm->ms[0] += sa;
    tm->ms[1] += sc;
    tm->launches[0] += ntimed;
    tm->launches[1] += ntimed;
    tm->bytes[0] += ntimed * b1;
    tm->bytes[1] += ntimed * b2;
    tm->launches_all += run;
    tm->ms_all[0] += sa / ntimed * run;
    tm->ms_all[1] += sc / ntimed * run;
    tm->bytes_all[0] += run * b1;
    tm->bytes_all[1] += run * b2;
    tm->split = true;
  }
}

// ---- fused block PCG of several problems --------------------------------
//
// Concurrent solves of a batch reach their inner CG at about the same time.
// Instead of one launch per problem and kernel, a group of CG calls with the
// same launch plan (element type, block width, step count, schedule and
// alignment; the sector dimensions may differ) runs as one launch per kernel:
// problem j owns a contiguous range of workgroups equal to its own grid, so
// it sums its rows in the same order as alone and gets the same bits.  The
// first caller of a group (the leader) waits a short time for peers, then
// enqueues the whole group's CG on its stream and the other callers' streams
// wait for it by events.

template <class T>
struct CgJob {
  const Ham* H;
  double sigma;
  const T* jac;
  const T* R;
  int64_t ldr;
  T* W;
  int64_t ldw;
  int b, m;
  bool aligned;
  Sched sc;
  T *r, *p, *t;
  double* part;
  PcgCoef* coef;
  hipStream_t s;
};

struct CgFuser {
  struct Ticket {
    void* job;
    hipEvent_t ready = nullptr, finished = nullptr;
    bool done = false;
    std::exception_ptr err;
  };
  // A group is open to new calls until it holds max_group of them or its
  // leader stops waiting; then it leaves `open`, and the next call with the
  // same key starts a new group.
  struct Group {
    std::vector<Ticket*> members;
    bool closed = false;
  };
  std::mutex mu;
  std::condition_variable cv;
  std::map<std::vector<int64_t>, std::shared_ptr<Group>> open;
  int max_group;
  std::chrono::microseconds wait;
  int64_t groups = 0, jobs = 0;
};

// the argument blocks of the fused kernels stay within the 4 KB kernel
// argument space
static_assert(sizeof(MultiApply<double>) <= 4096 && sizeof(MultiElt<double>) <= 4096 &&
                  sizeof(MultiFin) <= 4096,
              "fused kernel arguments too large");

template <class T>
void run_pcg_fused(const std::vector<CgJob<T>*>& g, hipStream_t s) {
  const int np = (int)g.size();
  if (np < 1 || np > kMaxFuse) fail(MBL_EINTERNAL, "fused pcg: group size out of range");
  const CgJob<T>& j0 = *g[0];
  const int b = j0.b, m = j0.m;
  for (const Chunk& ch : plan_chunks<T>(b, j0.aligned, j0.sc)) {
    std::vector<Grid> grid(np);
    MultiApply<T> m1{}, m2{};
    MultiElt<T> ei{}, eu{};
    MultiFin fin{};
    m1.np = m2.np = ei.np = eu.np = fin.np = np;
    int wg = 0;
    for (int k = 0; k < np; ++k) {
      const CgJob<T>& J = *g[k];
      const Grid gr = make_grid(J.H->n, ch.log2G, J.sc);
      m1.wg0[k] = m2.wg0[k] = ei.wg0[k] = eu.wg0[k] = wg;
      wg += (int)gr.nwg;
      ApplyArgs<T> a1 = base_args<T>(*J.H, J.sigma);  // T = (H - sigma) p, |T|^2
      a1.X = J.p;
      a1.ldx = b;
      a1.Y = J.t;
      a1.ldy = b;
      a1.part = J.part;
      ApplyArgs<T> a2 = base_args<T>(*J.H, J.sigma);  // q = (H - sigma) T, CG update
      a2.X = J.t;
      a2.ldx = b;
      a2.x = J.W;
      a2.ldxv = J.ldw;
      a2.r = J.r;
      a2.ldr = b;
      a2.p = J.p;
      a2.ldp = b;
      a2.jac = J.jac;
      a2.coef = J.coef;
      a2.part = J.part;
      for (ApplyArgs<T>* a : {&a1, &a2}) {
        a->col0 = ch.col0;
        a->w = ch.w;
        a->log2G = ch.log2G;
        a->ts = gr.ts;
      }
      m1.a[k] = a1;
      m2.a[k] = a2;
      EltArgs<T> e{};
      e.R = J.R;
      e.ldR = J.ldr;
      e.x = J.W;
      e.ldxv = J.ldw;
      e.r = J.r;
      e.ldr = b;
      e.p = J.p;
      e.ldp = b;
      e.jac = J.jac;
      e.coef = J.coef;
      e.part = J.part;
      e.n = J.H->n;
      e.col0 = ch.col0;
      e.w = ch.w;
      e.log2G = ch.log2G;
      e.ts = gr.ts;
      ei.a[k] = e;
      eu.a[k] = e;
      fin.c0[k] = k * ch.w;
      fin.part[k] = J.part;
      fin.nwg[k] = (int)gr.nwg;
      fin.col0[k] = ch.col0;
      fin.coef[k] = J.coef;
    }
    m1.wg0[np] = m2.wg0[np] = ei.wg0[np] = eu.wg0[np] = wg;
    fin.c0[np] = np * ch.w;
    const size_t red = (size_t)kWaves * ch.w * sizeof(double);
    const size_t shm = red + (size_t)kWaves * (64 >> ch.log2G) * 32 * sizeof(int) +
                       (MBL_APPLY_ALPHA_LDS ? (size_t)ch.w * sizeof(T) : 0);
    constexpr int VV = 16 / sizeof(T);
    auto launch_apply_multi = [&](const MultiApply<T>& ma, auto epi, hipStream_t st) {
      constexpr int EPI = decltype(epi)::value;
#define MBL_FUSE_CASE(VE_, NV_)                                                                 \
  if (ch.VE == VE_ && ch.NV == NV_) {                                                           \
    hipLaunchKernelGGL((k_apply_multi<T, VE_, NV_, EPI>), dim3(wg), dim3(kThreads), shm, st, ma); \
    MBL_CHECK_LAUNCH();                                                                         \
    return;                                                                                     \
  }
      MBL_FUSE_CASE(VV, 8)
      MBL_FUSE_CASE(VV, 4)
      MBL_FUSE_CASE(VV, 2)
      MBL_FUSE_CASE(VV, 1)
      MBL_FUSE_CASE(1, 4)
      MBL_FUSE_CASE(1, 2)
      MBL_FUSE_CASE(1, 1)
#undef MBL_FUSE_CASE
      fail(MBL_EINTERNAL, "fused pcg: no kernel for chunk shape");
    };
    auto launch_elt_multi = [&](const MultiElt<T>& me, auto mode, hipStream_t st) {
      constexpr int MODE = decltype(mode)::value;
      const size_t eshm = (MODE == ELT_INIT) ? red : 0;
#define MBL_FUSE_ELT(VE_, NV_)                                                                     \
  if (ch.VE == VE_ && ch.NV == NV_) {                                                              \
    hipLaunchKernelGGL((k_pcg_elt_multi<T, VE_, NV_, MODE>), dim3(wg), dim3(kThreads), eshm, st, me); \
    MBL_CHECK_LAUNCH();                                                                            \
    return;                                                                                        \
  }
      MBL_FUSE_ELT(VV, 8)
      MBL_FUSE_ELT(VV, 4)
      MBL_FUSE_ELT(VV, 2)
      MBL_FUSE_ELT(VV, 1)
      MBL_FUSE_ELT(1, 4)
      MBL_FUSE_ELT(1, 2)
      MBL_FUSE_ELT(1, 1)
#undef MBL_FUSE_ELT
      fail(MBL_EINTERNAL, "fused pcg: no kernel for chunk shape");
    };
    auto launch_fin = [&](auto mode, hipStream_t st) {
      constexpr int MODE = decltype(mode)::value;
      hipLaunchKernelGGL(k_pcg_finalize_multi<MODE>, dim3(np * ch.w), dim3(kThreads), 0, st, fin);
      MBL_CHECK_LAUNCH();
    };
    using E1 = std::integral_constant<int, EPI_NORM2>;
    using E2 = std::integral_constant<int, EPI_PCG>;
    using LI = std::integral_constant<int, ELT_INIT>;
    using LU = std::integral_constant<int, ELT_PUPD>;
    using FI = std::integral_constant<int, FIN_INIT>;
    using FA = std::integral_constant<int, FIN_ALPHA>;
    using FB = std::integral_constant<int, FIN_BETA>;
    launch_elt_multi(ei, LI{}, s);
    launch_fin(FI{}, s);
    auto step = [&]() {
      launch_apply_multi(m1, E1{}, s);
      launch_fin(FA{}, s);
      launch_apply_multi(m2, E2{}, s);
      launch_fin(FB{}, s);
      launch_elt_multi(eu, LU{}, s);
    };
    replay_steps(step, 0, m, s, nullptr);
  }
}

CgFuser* cg_fuser_create(int max_group, double wait_ms) {
  CgFuser* f = new CgFuser;
  f->max_group = std::max(1, std::min(max_group, kMaxFuse));
  f->wait = std::chrono::microseconds((int64_t)(1000.0 * std::max(0.0, wait_ms)));
  return f;
}

void cg_fuser_destroy(CgFuser* f) { delete f; }

void cg_fuser_stats(const CgFuser* f, int64_t* groups, int64_t* jobs) {
  *groups = f->groups;
  *jobs = f->jobs;
}

thread_local CgFuser* t_cg_fuser = nullptr;

// One CG call through the fuser: returns after the call's work (its own or
// its group's) is enqueued and `job.s` waits for it.
template <class T>
void fuse_pcg(CgFuser& f, CgJob<T>& job) {
  std::vector<int64_t> key = {(int64_t)sizeof(T), job.b, job.m, job.aligned ? 1 : 0,
                              job.sc.chunk_bytes, job.sc.lane_bytes, job.sc.grp, job.sc.slots};
  CgFuser::Ticket tk;
  tk.job = &job;
  MBL_HIP(hipEventCreateWithFlags(&tk.ready, hipEventDisableTiming));
  MBL_HIP(hipEventCreateWithFlags(&tk.finished, hipEventDisableTiming));
  struct Events {
    CgFuser::Ticket& t;
    ~Events() {
      (void)hipEventDestroy(t.ready);
      (void)hipEventDestroy(t.finished);
    }
  } ev{tk};
  MBL_HIP(hipEventRecord(tk.ready, job.s));  // R and the caller's buffers are ready
  std::unique_lock<std::mutex> lk(f.mu);
  std::shared_ptr<CgFuser::Group> grp;
  bool leader = false;
  auto it = f.open.find(key);
  if (it == f.open.end()) {
    grp = std::make_shared<CgFuser::Group>();
    f.open[key] = grp;
    leader = true;
  } else {
    grp = it->second;
  }
  grp->members.push_back(&tk);
  if ((int)grp->members.size() >= f.max_group) {  // full: no further call joins it
    grp->closed = true;
    f.open.erase(key);
    f.cv.notify_all();
  }
  if (!leader) {
    f.cv.wait(lk, [&] { return tk.done; });
  } else {
    // leader: gather peers for a short time, then run the group on this
    // caller's stream
    f.cv.wait_for(lk, f.wait, [&] { return grp->closed; });
    if (!grp->closed) {  // still the open group of this key
      grp->closed = true;
      f.open.erase(key);
    }
    const std::vector<CgFuser::Ticket*> members = grp->members;
    ++f.groups;
    f.jobs += (int64_t)members.size();
    lk.unlock();
    std::exception_ptr err;
    try {
      std::vector<CgJob<T>*> jobs;
      for (CgFuser::Ticket* t : members) {
        jobs.push_back(static_cast<CgJob<T>*>(t->job));
        if (t != &tk) MBL_HIP(hipStreamWaitEvent(job.s, t->ready, 0));
      }
      run_pcg_fused<T>(jobs, job.s);
      for (CgFuser::Ticket* t : members) MBL_HIP(hipEventRecord(t->finished, job.s));
    } catch (...) {
      err = std::current_exception();
    }
    lk.lock();
    for (CgFuser::Ticket* t : members) {
      t->err = err;
      t->done = true;
    }
    f.cv.notify_all();
  }
  lk.unlock();
  if (tk.err) std::rethrow_exception(tk.err);
  MBL_HIP(hipStreamWaitEvent(job.s, tk.finished, 0));
}

template <class T>
void run_pcg(const Ham& H, double sigma, const T* jac, const T* R, int64_t ldr, T* W, int64_t ldw,
             int b, int m, hipStream_t s, PcgTiming* tm, const StopCheck* stop, int keep,
             int m_keep) {
  const int64_t n = H.n;
  if (n == 0 || b == 0) return;
  const int wc = pcg_chunk_width<T>(n, b);
  if (t_cg_fuser && wc == b && keep < 0 && tm == nullptr && stop == nullptr && m >= 1) {
    // concurrent solves of a batch: this call may run in one launch with others
    CgJob<T> job{};
    job.sc = sched_for(H, b * (int)sizeof(T), (int)sizeof(T));
    job.aligned = al16(R, ldr, sizeof(T)) && al16(W, ldw, sizeof(T)) && (b * sizeof(T)) % 16 == 0;
    DevBuf rb((size_t)n * b * sizeof(T), s), pb((size_t)n * b * sizeof(T), s),
        tb((size_t)n * b * sizeof(T), s);
    DevBuf pa((size_t)kMaxWg * std::min(b, 4096) * sizeof(double) + 64, s);
    DevBuf cb((size_t)b * sizeof(PcgCoef), s);
    SplitCg<T> probe{W, ldw, rb.as<T>(), b, pb.as<T>(), b, tb.as<T>(), b, cb.as<PcgCoef>(),
                     pa.as<double>(), b};
    if (!split_cg_ready<T>(H, probe)) {
      job.H = &H;
      job.sigma = sigma;
      job.jac = jac;
      job.R = R;
      job.ldr = ldr;
      job.W = W;
      job.ldw = ldw;
      job.b = b;
      job.m = m;
      job.r = rb.as<T>();
      job.p = pb.as<T>();
      job.t = tb.as<T>();
      job.part = pa.as<double>();
      job.coef = cb.as<PcgCoef>();
      job.s = s;
      fuse_pcg<T>(*t_cg_fuser, job);
      return;
    }
  }
  DevBuf rbuf((size_t)n * wc * sizeof(T), s), pbuf((size_t)n * wc * sizeof(T), s),
      tbuf((size_t)n * wc * sizeof(T), s);
  DevBuf xbuf;
  if (wc < b) xbuf.reset((size_t)n * wc * sizeof(T), s);
  DevBuf part((size_t)kMaxWg * std::min(wc, 4096) * sizeof(double) + 64, s);
  DevBuf coefb((size_t)b * sizeof(PcgCoef), s);
  T* r = rbuf.as<T>();
  T* p = pbuf.as<T>();
  T* t = tbuf.as<T>();
  PcgCoef* coef = coefb.as<PcgCoef>();
  for (int c0 = 0; c0 < b; c0 += wc) {
    const int w = std::min(wc, b - c0);
    // chunk views: inputs/outputs of the caller, compact CG vectors (ld = w)
    const T* Rc = R + c0;
    T* x = (wc < b) ? xbuf.as<T>() : W;
    const int64_t ldx = (wc < b) ? w : ldw;
    PcgCoef* cf = coef + c0;
    const bool aligned = al16(Rc, ldr, sizeof(T)) && al16(x, ldx, sizeof(T)) && al16(r, w, sizeof(T));
    const Sched sc = sched_for(H, w * (int)sizeof(T), (int)sizeof(T));
    SplitCg<T> sg{x, ldx, r, w, p, w, t, w, cf, part.as<double>(), w};
    if (split_cg_ready<T>(H, sg)) {
      run_pcg_split<T>(H, sigma, jac, Rc, ldr, sg, std::max(m, m_keep), aligned, sc, s, tm, stop);
      if (wc < b)
        MBL_HIP(hipMemcpy2DAsync(W + c0, ldw * sizeof(T), x, w * sizeof(T), w * sizeof(T), n,
                                 hipMemcpyDeviceToDevice, s));
      continue;
    }
    // CG steps [from, to) on the columns of chunk ch (events on the first
    // timed steps of the solve's first pass over the chunk)
    auto cg_steps = [&](const Chunk& ch, const Sched& sch, int from, int to, bool timed) {
      const Grid g = make_grid(n, ch.log2G, sch);
      EltArgs<T> e{};
      e.x = x;
      e.ldxv = ldx;
      e.r = r;
      e.ldr = w;
      e.p = p;
      e.ldp = w;
      e.jac = jac;
      e.coef = cf;
      e.part = part.as<double>();
      e.n = n;
      ApplyArgs<T> a1 = base_args<T>(H, sigma);  // T = (H - sigma) p, |T|^2
      a1.X = p;
      a1.ldx = w;
      a1.Y = t;
      a1.ldy = w;
      a1.part = part.as<double>();
      ApplyArgs<T> a2 = base_args<T>(H, sigma);  // q = (H - sigma) T, CG update
      a2.X = t;
      a2.ldx = w;
      a2.x = x;
      a2.ldxv = ldx;
      a2.r = r;
      a2.ldr = w;
      a2.p = p;
      a2.ldp = w;
      a2.jac = jac;
      a2.coef = cf;
      a2.part = part.as<double>();
      const int ntimed = (tm && timed) ? std::min(to - from, PcgTiming::kSample) : 0;
      if (ntimed) tm->init();
      auto step = [&]() {
        dispatch_apply<T, EPI_NORM2>(ch, g, a1, s);
        finalize<FIN_ALPHA>(ch, g, part.as<double>(), cf, s);
        dispatch_apply<T, EPI_PCG>(ch, g, a2, s);
        finalize<FIN_BETA>(ch, g, part.as<double>(), cf, s);
        dispatch_elt<T, ELT_PUPD>(ch, g, e, s);
      };
      int it = from;
      for (int k = 0; k < ntimed; ++k, ++it) {
        MBL_HIP(hipEventRecord(tm->ev[4 * k + 0], s));
        dispatch_apply<T, EPI_NORM2>(ch, g, a1, s);
        MBL_HIP(hipEventRecord(tm->ev[4 * k + 1], s));
        finalize<FIN_ALPHA>(ch, g, part.as<double>(), cf, s);
        MBL_HIP(hipEventRecord(tm->ev[4 * k + 2], s));
        dispatch_apply<T, EPI_PCG>(ch, g, a2, s);
        MBL_HIP(hipEventRecord(tm->ev[4 * k + 3], s));
        finalize<FIN_BETA>(ch, g, part.as<double>(), cf, s);
        dispatch_elt<T, ELT_PUPD>(ch, g, e, s);
      }
      // The remaining steps replay one captured step: every CG coefficient
      // lives on the device, so the five launches are identical each step.
      const int run = replay_steps(step, it, to, s, stop) - from;
      if (ntimed > 0) {
        MBL_HIP(hipStreamSynchronize(s));
        double sa = 0.0, sc = 0.0;
        for (int k = 0; k < ntimed; ++k) {
          float ta = 0.f, tc = 0.f;
          MBL_HIP(hipEventElapsedTime(&ta, tm->ev[4 * k + 0], tm->ev[4 * k + 1]));
          MBL_HIP(hipEventElapsedTime(&tc, tm->ev[4 * k + 2], tm->ev[4 * k + 3]));
          sa += ta;
          sc += tc;
        }
        const double b1 = 2.0 * n * ch.w * sizeof(T) + 12.0 * n;
        const double b2 = 6.0 * n * ch.w * sizeof(T) + (12.0 + sizeof(T)) * n;
        tm->ms[0] += sa;
        tm->ms[1] += sc;
        tm->launches[0] += ntimed;
        tm->launches[1] += ntimed;
        tm->bytes[0] += ntimed * b1;
        tm->bytes[1] += ntimed * b2;
        tm->launches_all += run;
        tm->ms_all[0] += sa / ntimed * run;
        tm->ms_all[1] += sc / ntimed * run;
        tm->bytes_all[0] += run * b1;
        tm->bytes_all[1] += run * b2;
      }
    };
    for (const Chunk& ch : plan_chunks<T>(w, aligned, sc)) {
      if ((size_t)ch.w * kMaxWg * sizeof(double) > part.bytes()) fail(MBL_EINTERNAL, "pcg: part");
      {
        const Grid g = make_grid(n, ch.log2G, sc);
        EltArgs<T> e{};
        e.R = Rc;
        e.ldR = ldr;
        e.x = x;
        e.ldxv = ldx;
        e.r = r;
        e.ldr = w;
        e.p = p;
        e.ldp = w;
        e.jac = jac;
        e.coef = cf;
        e.part = part.as<double>();
        e.n = n;
        dispatch_elt<T, ELT_INIT>(ch, g, e, s);
        finalize<FIN_INIT>(ch, g, part.as<double>(), cf, s);
      }
      // columns [0, keep) of the whole block run m_keep steps, the others m
      const int lo = c0 + ch.col0, hi = lo + ch.w;
      if (hi <= keep || m_keep <= m) {
        cg_steps(ch, sc, 0, hi <= keep ? std::max(m, m_keep) : m, true);
      } else {
        cg_steps(ch, sc, 0, m, true);
        if (lo < keep) {
          // the leading columns of this chunk go on (same vectors and ld),
          // under the schedule tuned for their own row width
          const Sched sk = sched_for(H, (keep - lo) * (int)sizeof(T), (int)sizeof(T));
          for (const Chunk& sub : plan_chunks<T>(keep - lo, aligned, sk)) {
            Chunk c2 = sub;
            c2.col0 += ch.col0;
            cg_steps(c2, sk, m, m_keep, true);
          }
        }
      }
    }
    if (wc < b)
      MBL_HIP(hipMemcpy2DAsync(W + c0, ldw * sizeof(T), x, w * sizeof(T), w * sizeof(T), n,
                               hipMemcpyDeviceToDevice, s));
  }
}

template void launch_apply<double>(const Ham&, double, const double*, int64_t, double*, int64_t,
                                   int, hipStream_t);
template void launch_apply<float>(const Ham&, double, const float*, int64_t, float*, int64_t, int,
                                  hipStream_t);
template void run_pcg<double>(const Ham&, double, const double*, const double*, int64_t, double*,
                              int64_t, int, int, hipStream_t, PcgTiming*, const StopCheck*, int,
                              int);
template void run_pcg<float>(const Ham&, double, const float*, const float*, int64_t, float*,
                             int64_t, int, int, hipStream_t, PcgTiming*, const StopCheck*, int,
                             int);

}  // namespace mbl
