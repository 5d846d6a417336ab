// Two-pass (split) matrix-free apply Y = (H - sigma I) X and the fused CG
// steps built from it (paper Sec. 3.2 and 4.1).
//
// Why two passes.  Every row has about L/2 active flip-flop bonds whose
// targets sit at +-C(i, t) rows (colex order); for the high bonds those are
// millions of rows away, so a one-pass gather re-reads rows that have left
// the 4 MB L2 of the XCD.  Here the chain is cut between sites q-1 and q
// (q = L/2); a state is s = (hi << q) | lo.  In row order the rows with one
// fixed hi are a contiguous block indexed by the colex rank of lo, and a flip
// inside the low half moves within that block (by the same +-C(i, t) rule,
// applied to lo), while a flip inside the high half keeps lo and moves hi.
//   high pass: a tile is one lo configuration with every hi it combines
//              with (C(L-q, k_hi) rows, one per block); it stages those rows
//              (one column panel) in LDS and gathers the high-half flips
//              there.
//   low pass:  a tile is one block (C(q, k_lo) consecutive rows); it stages
//              them in LDS, gathers the low-half flips there, adds the
//              diagonal and the middle bond (q-1, q) -- whose target is in the
//              neighbouring block hi ^ 1, read from memory, usually from the
//              L2 since that block is processed beside it -- and the high
//              pass's partial result.
// So every row of X is read from memory about twice and no gather leaves
// LDS, at the price of writing and re-reading one partial result.
//
// The diagonal E(s) = E_lo(lo) + E_hi(hi) + E_mid and the anti-aligned bond
// count (for the Jacobi diagonal (E - sigma)^2 + (J/2)^2 nd) come from per-half
// tables of 2^q and 2^(L-q) entries, so no n-length table is read.
//
// CG steps (per column, Jacobi-PCG on (H - sigma)^2, see apply.hip):
//   apply1: high pass with the p-update fused into its load phase
//           (p = M^-1 r + beta p on the tile's rows, written back), low pass
//           with |T|^2 partial sums;
//   apply2: high pass subtracts alpha (high part of (H - sigma) T) from r and
//           does x += alpha p, low pass subtracts the rest and forms the
//           r.M^-1 r partial sums.
//
// Work distribution: persistent grid of 8 x slots x panels workgroups;
// workgroup k runs on XCD k % 8 and takes a contiguous range of the tile list
// (balanced by rows), so a block and its middle-bond neighbour are processed
// by the same XCD at about the same time; the panels of one tile run side by
// side on that XCD and share its cache lines.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "common.h"

namespace mbl {

namespace {

#ifndef MBL_SPLIT_THREADS
#define MBL_SPLIT_THREADS 512
#endif
#ifndef MBL_SPLIT_TILE_BYTES
#define MBL_SPLIT_TILE_BYTES 32768
#endif
constexpr int kSpThreads = MBL_SPLIT_THREADS;
constexpr int kSpWaves = kSpThreads / 64;
constexpr int kSpC = 17;  // C(i, t) for i, t <= 16: a half chain has at most 16 sites
constexpr int kSpCBytes = ((kSpC * kSpC * 4 + 15) / 16) * 16;

template <class T, int VE>
struct alignas(sizeof(T) * VE) SVec {
  T v[VE];
};

template <class T, int VE>
__device__ inline SVec<T, VE> vload(const T* p) {
  return *reinterpret_cast<const SVec<T, VE>*>(p);
}

template <class T, int VE>
__device__ inline void vstore_nt(T* p, const SVec<T, VE>& v) {
  typedef T vec_t __attribute__((ext_vector_type(VE)));
  vec_t x;
#pragma unroll
  for (int e = 0; e < VE; ++e) x[e] = v.v[e];
  __builtin_nontemporal_store(x, reinterpret_cast<vec_t*>(p));
}

enum { PASS_LOW = 0, PASS_HIGH = 1 };
enum { EP_PLAIN = 0, EP_PUPD = 1, EP_RUPD = 2, EP_NORM2 = 3, EP_PCG = 4 };

template <class T>
struct SplitArgs {
  const SplitTile* tiles;
  const uint32_t* info;    // lo_info (low pass) / hi_info (high pass)
  const double* Etab;      // lo_E / hi_E
  const uint32_t* hoff;    // high pass: first row of each hi's block
  const uint32_t* pascal;  // 33 x 33
  const T* X;
  int64_t ldx;
  T* Y;
  int64_t ldy;
  T* x;
  int64_t ldxv;
  T* r;
  int64_t ldr;
  T* p;
  int64_t ldp;
  const PcgCoef* coef;
  double* part;
  int64_t n;
  double sigma, halfJ, zz4;
  int q, nb;  // cut position; bonds inside this pass's half
  int maxrows;  // rows of the LDS tile (the middle-bond rows follow it)
  int w, log2G, npanels, nslots;
  int xcd_first[9];
};

// Rows of one tile per thread: the host picks the panel width so that
// maxrows * panel bytes <= 32 KB, i.e. maxrows <= 4 * (rows per workgroup pass).
constexpr int kRowsPerThread = 4;
constexpr size_t kTileBytes = MBL_SPLIT_TILE_BYTES;

// Asynchronous copy of 16 bytes per lane from global memory into LDS: lane l of
// the wavefront writes lds_base + 16 l.  lds_base must be the same in every
// lane; lanes that are switched off copy nothing.
template <class T>
__device__ inline void dma16(const T* g, T* lds_base) {
  __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(g),
                                   reinterpret_cast<__attribute__((address_space(3))) void*>(
                                       reinterpret_cast<uintptr_t>(lds_base)),
                                   16, 0, 0);
}

// Thread layout: G = 2^log2G lanes per tile row, 16 bytes each (one panel row
// = 16 G bytes); RW = 64 / G consecutive rows per wavefront and RPI = 512 / G
// rows per workgroup pass, so the wave's lanes cover one contiguous slab of the
// LDS tile and the copy engine's lane order is the tile's layout.  Thread
// (wave w, lane l) owns rows u_k = k RPI + w RW + l / G, k < 8.
template <class T, int PASS, int EPI>
__global__ __launch_bounds__(kSpThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_split(SplitArgs<T> a) {
  constexpr int VE = 16 / (int)sizeof(T);
  using P = SVec<T, VE>;
  constexpr bool kRed = (EPI == EP_NORM2 || EPI == EP_PCG);
  constexpr int KR = kRowsPerThread;
  extern __shared__ __align__(16) unsigned char smem[];
  uint32_t* C = reinterpret_cast<uint32_t*>(smem);
  const int G = 1 << a.log2G;
  const int PBe = G * VE;  // elements of one panel row
  double* sred = reinterpret_cast<double*>(smem + kSpCBytes);
  T* tile = reinterpret_cast<T*>(smem + kSpCBytes + (kRed ? kSpWaves * PBe * 8 : 0));
  T* mtile = tile + (size_t)a.maxrows * PBe;  // low pass: middle-bond rows
  for (int i = threadIdx.x; i < kSpC * kSpC; i += kSpThreads)
    C[i] = a.pascal[(i / kSpC) * kPascal + (i % kSpC)];

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int RW = 64 >> a.log2G;
  const int RPI = kSpThreads >> a.log2G;
  const int cl = threadIdx.x & (G - 1), rsub = threadIdx.x >> a.log2G;
  const int xcd = blockIdx.x & 7, rest = blockIdx.x >> 3;
  const int panel = rest % a.npanels, slot = rest / a.npanels;
  const int col = panel * PBe + cl * VE;  // this lane's first column
  const bool act = col < a.w;             // w is a multiple of VE
  T alpha[VE], beta[VE];
  bool live[VE];
#pragma unroll
  for (int e = 0; e < VE; ++e) {
    alpha[e] = (T)0;
    beta[e] = (T)0;
    live[e] = false;
  }
  if (act) {
    if constexpr (EPI == EP_RUPD || EPI == EP_PCG) {
#pragma unroll
      for (int e = 0; e < VE; ++e) alpha[e] = (T)a.coef[col + e].alpha;
    }
    if constexpr (EPI == EP_PUPD) {
#pragma unroll
      for (int e = 0; e < VE; ++e) {
        beta[e] = (T)a.coef[col + e].beta;
        live[e] = a.coef[col + e].live != 0;
      }
    }
  }
  double red[VE];
#pragma unroll
  for (int e = 0; e < VE; ++e) red[e] = 0.0;
  const T hj = (T)a.halfJ;
  const int nbm = a.nb > 0 ? a.nb : 0;
  const uint32_t bmask = nbm > 0 ? ((1u << nbm) - 1u) : 0u;
  (void)lane;
  __syncthreads();

  const int tb = a.xcd_first[xcd], te = a.xcd_first[xcd + 1];
  for (int t = tb + slot; t < te; t += a.nslots) {
    const SplitTile tl = a.tiles[t];
    const int nr = tl.nrows;
    const uint32_t fixed = tl.code;  // the half that is constant over the tile
    // Per row u_k of this thread, kept across the barrier: the varying half's
    // configuration, the row (high pass), the part of the result that needs
    // no LDS gather, and the diagonal factors.
    uint32_t infok[KR];
    int32_t rowk[KR];
    T part[KR][VE];
    T edk[KR], dinvk[KR];
    // 1. low pass: own rows (consecutive) and the middle-bond targets (a
    //    consecutive slice of the block hi ^ 1) straight into LDS; the middle
    //    row of tile row u goes to mtile[u - mlo]
    const int mlo = (fixed & 1u) ? 0 : tl.msplit;
    if constexpr (PASS == PASS_LOW) {
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        const int u = rsub + k * RPI;
        if (act && u < nr) {
          dma16<T>(a.X + ((int64_t)tl.row0 + u) * a.ldx + col,
                   tile + (size_t)(k * RPI + wave * RW) * PBe);
          const bool midrow = (fixed & 1u) ? (u < tl.msplit) : (u >= tl.msplit);
          if (midrow)
            dma16<T>(a.X + (int64_t)(tl.mbase + u) * a.ldx + col,
                     mtile + (ptrdiff_t)(k * RPI + wave * RW - mlo) * PBe);
        }
      }
    }
    // 2. tables: configuration, row (high pass), diagonal factors
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int u = rsub + k * RPI;
      const bool ok = act && u < nr;
      infok[k] = ok ? a.info[tl.aux + u] : 0u;
      if constexpr (PASS == PASS_LOW)
        rowk[k] = tl.row0 + u;
      else
        rowk[k] = ok ? (int32_t)a.hoff[tl.aux + u] + tl.row0 : 0;
      edk[k] = dinvk[k] = (T)0;
      if constexpr (PASS == PASS_LOW || EPI == EP_PUPD) {
        if (ok) {
          // same sum and order as the diagonal kernel
          const double Et = a.Etab[tl.aux + u];
          const uint32_t li = (PASS == PASS_LOW) ? infok[k] : fixed;
          const uint32_t hii = (PASS == PASS_LOW) ? fixed : infok[k];
          const double El = (PASS == PASS_LOW) ? Et : tl.E;
          const double Eh = (PASS == PASS_LOW) ? tl.E : Et;
          const uint32_t lo = li & 0xFFFFFFu, hi = hii & 0xFFFFFFu;
          const bool mid = (((lo >> (a.q - 1)) ^ hi) & 1u) != 0;
          const double e0 = ((El + Eh) + (mid ? -a.zz4 : a.zz4)) - a.sigma;
          const int nd = (int)(li >> 24) + (int)(hii >> 24) + (mid ? 1 : 0);
          edk[k] = (T)e0;
          if constexpr (EPI == EP_PUPD || EPI == EP_PCG)
            dinvk[k] = (T)1 / (T)(e0 * e0 + a.halfJ * a.halfJ * (double)nd);
        }
      }
    }
    // 3. high pass: own rows into LDS (after the p-update for apply1)
    if constexpr (PASS == PASS_HIGH && EPI != EP_PUPD) {
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        const int u = rsub + k * RPI;
        if (act && u < nr)
          dma16<T>(a.X + (int64_t)rowk[k] * a.ldx + col, tile + (size_t)(k * RPI + wave * RW) * PBe);
      }
    }
    // 4. epilogue operands, folded into part[] as they arrive
    {
      P av[KR], bv[KR];
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        const int u = rsub + k * RPI;
#pragma unroll
        for (int e = 0; e < VE; ++e) av[k].v[e] = bv[k].v[e] = (T)0;
        if (!(act && u < nr)) continue;
        const int64_t row = rowk[k];
        if constexpr (PASS == PASS_LOW) {
          if constexpr (EPI == EP_PLAIN || EPI == EP_NORM2)
            av[k] = vload<T, VE>(a.Y + row * a.ldy + col);  // the high pass's part
          else
            av[k] = vload<T, VE>(a.r + row * a.ldr + col);
        } else if constexpr (EPI == EP_RUPD) {
          av[k] = vload<T, VE>(a.r + row * a.ldr + col);
        } else if constexpr (EPI == EP_PUPD) {
          av[k] = vload<T, VE>(a.r + row * a.ldr + col);
          bv[k] = vload<T, VE>(a.p + row * a.ldp + col);
        }
      }
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        const int u = rsub + k * RPI;
#pragma unroll
        for (int e = 0; e < VE; ++e) part[k][e] = (T)0;
        if (!(act && u < nr)) continue;
        if constexpr (PASS == PASS_LOW || EPI == EP_RUPD) {
#pragma unroll
          for (int e = 0; e < VE; ++e) part[k][e] = av[k].v[e];
        } else if constexpr (EPI == EP_PUPD) {
          // p = M^-1 r + beta p (live columns): to memory and to the LDS tile
          P pv = bv[k];
#pragma unroll
          for (int e = 0; e < VE; ++e)
            if (live[e]) pv.v[e] = av[k].v[e] * dinvk[k] + beta[e] * pv.v[e];
          vstore_nt<T, VE>(a.p + (int64_t)rowk[k] * a.ldp + col, pv);
          *reinterpret_cast<P*>(tile + (size_t)u * PBe + cl * VE) = pv;
        }
      }
    }
    if constexpr (EPI == EP_RUPD) {
      // x += alpha p on this thread's rows, four at a time
#pragma unroll
      for (int h = 0; h < KR; h += 4) {
        P pv[4], xv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int u = rsub + (h + j) * RPI;
          if (act && u < nr) {
            pv[j] = vload<T, VE>(a.p + (int64_t)rowk[h + j] * a.ldp + col);
            xv[j] = vload<T, VE>(a.x + (int64_t)rowk[h + j] * a.ldxv + col);
          }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int u = rsub + (h + j) * RPI;
          if (act && u < nr) {
#pragma unroll
            for (int e = 0; e < VE; ++e) xv[j].v[e] = xv[j].v[e] + alpha[e] * pv[j].v[e];
            vstore_nt<T, VE>(a.x + (int64_t)rowk[h + j] * a.ldxv + col, xv[j]);
          }
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0);  // this wavefront's LDS copies have landed
    __syncthreads();
    // 5. flips inside the half from LDS, then the stores
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int u = rsub + k * RPI;
      if (!(act && u < nr)) continue;
      const uint32_t bits = infok[k] & 0xFFFFFFu;
      T acc[VE];
#pragma unroll
      for (int e = 0; e < VE; ++e) acc[e] = (T)0;
      uint32_t m = (bits ^ (bits >> 1)) & bmask;  // active bonds of this half
      while (m) {
        const int i = __ffs(m) - 1;
        m &= m - 1u;
        const int c = (int)C[i * kSpC + __popc(bits & ((1u << i) - 1u))];
        const int u2 = ((bits >> i) & 1u) ? u + c : u - c;
        if (u2 >= 0 && u2 < nr) {  // always true for a valid table
          const P g = *reinterpret_cast<const P*>(tile + (size_t)u2 * PBe + cl * VE);
#pragma unroll
          for (int e = 0; e < VE; ++e) acc[e] += g.v[e];
        }
      }
      const int64_t row = rowk[k];
      P o;
      if constexpr (PASS == PASS_LOW) {
        const bool midrow = (fixed & 1u) ? (u < tl.msplit) : (u >= tl.msplit);
        if (midrow) {
          const P g = *reinterpret_cast<const P*>(mtile + (size_t)(u - mlo) * PBe + cl * VE);
#pragma unroll
          for (int e = 0; e < VE; ++e) acc[e] += g.v[e];
        }
        const P own = *reinterpret_cast<const P*>(tile + (size_t)u * PBe + cl * VE);
        if constexpr (EPI == EP_PLAIN || EPI == EP_NORM2) {
#pragma unroll
          for (int e = 0; e < VE; ++e) o.v[e] = part[k][e] + (edk[k] * own.v[e] + hj * acc[e]);
          vstore_nt<T, VE>(a.Y + row * a.ldy + col, o);
          if constexpr (EPI == EP_NORM2) {
#pragma unroll
            for (int e = 0; e < VE; ++e) red[e] += (double)o.v[e] * (double)o.v[e];
          }
        } else {
#pragma unroll
          for (int e = 0; e < VE; ++e) {
            o.v[e] = part[k][e] - alpha[e] * (edk[k] * own.v[e] + hj * acc[e]);
            red[e] += (double)o.v[e] * (double)(o.v[e] * dinvk[k]);
          }
          vstore_nt<T, VE>(a.r + row * a.ldr + col, o);
        }
      } else {  // PASS_HIGH
        if constexpr (EPI == EP_RUPD) {
#pragma unroll
          for (int e = 0; e < VE; ++e) o.v[e] = part[k][e] - alpha[e] * (hj * acc[e]);
          vstore_nt<T, VE>(a.r + row * a.ldr + col, o);
        } else {
#pragma unroll
          for (int e = 0; e < VE; ++e) o.v[e] = hj * acc[e];
          vstore_nt<T, VE>(a.Y + row * a.ldy + col, o);
        }
      }
    }
    __syncthreads();  // the next tile's copies overwrite the LDS tile
  }

  if constexpr (kRed) {
    // fixed-order reduction: lanes of one column within the wavefront
    // (butterfly), then the waves in order; one partial per workgroup
#pragma unroll
    for (int e = 0; e < VE; ++e)
      for (int off = G; off < 64; off <<= 1) red[e] += __shfl_xor(red[e], off);
    if ((threadIdx.x & 63) < G) {
#pragma unroll
      for (int e = 0; e < VE; ++e) sred[wave * PBe + cl * VE + e] = red[e];
    }
    __syncthreads();
    const int nwp = 8 * a.nslots;
    for (int c = threadIdx.x; c < PBe; c += kSpThreads) {
      if (panel * PBe + c >= a.w) continue;
      double s = sred[c];
      for (int wv = 1; wv < kSpWaves; ++wv) s += sred[wv * PBe + c];
      a.part[(int64_t)(panel * PBe + c) * nwp + (xcd * a.nslots + slot)] = s;
    }
  }
}

int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v ? std::atoi(v) : dflt;
}

struct SplitPlan {
  int pb = 0, log2G = 0, npanels = 0, nslots = 0;
  size_t lds[2][2] = {};  // [pass][with reduction]
};

// LDS bytes: Pascal table, reduction scratch (one FP64 per panel column and
// wave, sized for 4-byte elements), the tile and (low pass) the middle-bond rows.
size_t split_lds(int rows, int mid, int pb, bool red) {
  return (size_t)kSpCBytes + (red ? (size_t)kSpWaves * (pb / 4) * 8 : 0) + (size_t)(rows + mid) * pb;
}

// Panel width: the widest of 256 ... 16 bytes that is not wider than the row
// and whose largest tile fits kTileBytes (so that every thread holds at most
// kRowsPerThread rows).  MBL_SPLIT_PANEL_BYTES forces a width (still checked).
bool make_plan(const Ham& H, int row_bytes, SplitPlan* pl) {
  const SplitTables& S = H.split;
  if (!S.ok || row_bytes < 16 || row_bytes % 16 != 0) return false;
  const int mr = std::max(S.maxrows[0], S.maxrows[1]);
  const int forced = env_int("MBL_SPLIT_PANEL_BYTES", 0);
  int pb = 0;
  for (int c = 256; c >= 16; c >>= 1) {
    if (forced > 0 && c != forced) continue;
    if (c > row_bytes && !(forced > 0)) continue;
    if ((size_t)mr * c <= kTileBytes) {
      pb = c;
      break;
    }
  }
  if (pb == 0) return false;
  int log2G = 0;
  while ((16 << log2G) < pb) ++log2G;
  if (mr > kRowsPerThread * (kSpThreads >> log2G)) return false;
  pl->pb = pb;
  pl->log2G = log2G;
  pl->npanels = (row_bytes + pb - 1) / pb;
  for (int ps = 0; ps < 2; ++ps)
    for (int rd = 0; rd < 2; ++rd)
      pl->lds[ps][rd] = split_lds(S.maxrows[ps], ps == PASS_LOW ? S.maxmid : 0, pb, rd != 0);
  const size_t worst = std::max(pl->lds[0][1], pl->lds[1][1]);
  const int per_cu =
      (int)std::max<size_t>(1, std::min<size_t>(2048 / kSpThreads, (160 * 1024) / worst));
  const int dflt = std::max(1, 32 * per_cu / pl->npanels);
  pl->nslots = std::max(1, std::min(256, env_int("MBL_SPLIT_SLOTS", dflt)));
  return true;
}

template <class T>
SplitArgs<T> split_args(const Ham& H, double sigma, const SplitPlan& pl, int pass, int w) {
  const SplitTables& S = H.split;
  SplitArgs<T> a{};
  a.tiles = S.tiles[pass].as<SplitTile>();
  a.info = (pass == PASS_LOW ? S.lo_info : S.hi_info).as<uint32_t>();
  a.Etab = (pass == PASS_LOW ? S.lo_E : S.hi_E).as<double>();
  a.hoff = S.hoff.as<uint32_t>();
  a.pascal = H.pascal.as<uint32_t>();
  a.n = H.n;
  a.sigma = sigma;
  a.halfJ = 0.5 * H.J;
  a.zz4 = 0.25 * H.J * H.Delta;
  a.q = S.q;
  a.nb = (pass == PASS_LOW) ? S.q - 1 : S.Lh - 1;
  a.maxrows = S.maxrows[pass];
  a.w = w;
  a.log2G = pl.log2G;
  a.npanels = pl.npanels;
  a.nslots = pl.nslots;
  for (int i = 0; i < 9; ++i) a.xcd_first[i] = S.xcd_first[pass][i];
  return a;
}

template <class T, int PASS, int EPI>
void launch_pass(const SplitPlan& pl, const SplitArgs<T>& a, hipStream_t s) {
  constexpr bool red = (EPI == EP_NORM2 || EPI == EP_PCG);
  const size_t shm = pl.lds[PASS][red ? 1 : 0];
  const unsigned nwg = (unsigned)(8 * pl.nslots * pl.npanels);
  hipLaunchKernelGGL((k_split<T, PASS, EPI>), dim3(nwg), dim3(kSpThreads), shm, s, a);
  MBL_CHECK_LAUNCH();
}

bool al16(const void* p, int64_t ld, size_t es) {
  return (reinterpret_cast<uintptr_t>(p) % 16 == 0) && ((ld * (int64_t)es) % 16 == 0);
}

}  // namespace

bool split_usable(const Ham& H, int row_bytes) {
  // Off unless MBL_APPLY_SPLIT=1: on the MI355X the one-pass kernel is faster
  // at every workload size (its re-reads are mostly served by the last-level
  // cache, while these passes stream at the plain copy rate).
  if (env_int("MBL_APPLY_SPLIT", 0) != 1 || !H.split.ok) return false;
  SplitPlan pl;
  return make_plan(H, row_bytes, &pl);
}

template <class T>
bool split_apply(const Ham& H, double sigma, const T* X, int64_t ldx, T* Y, int64_t ldy, int w,
                 hipStream_t s) {
  if (H.n == 0 || w == 0) return true;
  if (!split_usable(H, w * (int)sizeof(T))) return false;
  if (!al16(X, ldx, sizeof(T)) || !al16(Y, ldy, sizeof(T))) return false;
  SplitPlan pl;
  make_plan(H, w * (int)sizeof(T), &pl);
  SplitArgs<T> hi = split_args<T>(H, sigma, pl, PASS_HIGH, w);
  hi.X = X;
  hi.ldx = ldx;
  hi.Y = Y;
  hi.ldy = ldy;
  launch_pass<T, PASS_HIGH, EP_PLAIN>(pl, hi, s);
  SplitArgs<T> lo = split_args<T>(H, sigma, pl, PASS_LOW, w);
  lo.X = X;
  lo.ldx = ldx;
  lo.Y = Y;  // in place: each row's high part is read and overwritten by one thread
  lo.ldy = ldy;
  launch_pass<T, PASS_LOW, EP_PLAIN>(pl, lo, s);
  return true;
}

template <class T>
bool split_cg_ready(const Ham& H, const SplitCg<T>& c) {
  if (!split_usable(H, c.w * (int)sizeof(T))) return false;
  return al16(c.x, c.ldx, sizeof(T)) && al16(c.r, c.ldr, sizeof(T)) &&
         al16(c.p, c.ldp, sizeof(T)) && al16(c.t, c.ldt, sizeof(T));
}

template <class T>
int split_cg_apply(const Ham& H, double sigma, int op, const SplitCg<T>& c, hipStream_t s) {
  SplitPlan pl;
  if (!make_plan(H, c.w * (int)sizeof(T), &pl)) fail(MBL_EINTERNAL, "split CG: no plan");
  SplitArgs<T> hi = split_args<T>(H, sigma, pl, PASS_HIGH, c.w);
  SplitArgs<T> lo = split_args<T>(H, sigma, pl, PASS_LOW, c.w);
  for (SplitArgs<T>* a : {&hi, &lo}) {
    a->x = c.x;
    a->ldxv = c.ldx;
    a->r = c.r;
    a->ldr = c.ldr;
    a->p = c.p;
    a->ldp = c.ldp;
    a->coef = c.coef;
    a->part = c.part;
  }
  if (op == 0) {
    // p = M^-1 r + beta p (live columns), T = (H - sigma) p, |T|^2
    hi.Y = c.t;
    hi.ldy = c.ldt;
    launch_pass<T, PASS_HIGH, EP_PUPD>(pl, hi, s);
    lo.X = c.p;
    lo.ldx = c.ldp;
    lo.Y = c.t;
    lo.ldy = c.ldt;
    launch_pass<T, PASS_LOW, EP_NORM2>(pl, lo, s);
  } else {
    // q = (H - sigma) T: r -= alpha q (high part, then the rest), x += alpha p
    hi.X = c.t;
    hi.ldx = c.ldt;
    launch_pass<T, PASS_HIGH, EP_RUPD>(pl, hi, s);
    lo.X = c.t;
    lo.ldx = c.ldt;
    launch_pass<T, PASS_LOW, EP_PCG>(pl, lo, s);
  }
  return 8 * pl.nslots;
}

// ---- tables (host) ----------------------------------------------------------

void build_split_tables(Ham& H, hipStream_t s) {
  SplitTables& S = H.split;
  const int L = H.L, k = H.nup;
  const int q = L / 2, Lh = L - q;
  S.q = q;
  S.Lh = Lh;
  S.ok = false;
  S.maxmid = 0;
  if (L < 2 || q > 16 || Lh > 16) return;
  const auto& Cp = H.pascal_host;
  auto Cb = [&](int i, int t) -> int64_t { return (t < 0 || t > i) ? 0 : Cp[i * kPascal + t]; };
  const double zz4 = 0.25 * H.J * H.Delta;
  // energy and anti-aligned bond count of a half (len sites from site base)
  auto half = [&](int base, int len, uint32_t v, int* nd) {
    double e = 0.0;
    int c = 0;
    for (int i = 0; i + 1 < len; ++i) {
      const bool anti = (((v >> i) ^ (v >> (i + 1))) & 1u) != 0;
      e += anti ? -zz4 : zz4;
      c += anti ? 1 : 0;
    }
    for (int i = 0; i < len; ++i) e += H.h[base + i] * (((v >> i) & 1u) ? 0.5 : -0.5);
    *nd = c;
    return e;
  };
  // configurations of a half sorted by (up spins, value), with the start of
  // each up-spin count
  auto sorted = [&](int len, std::vector<uint32_t>& vals, std::vector<int>& base) {
    const uint32_t N = 1u << len;
    base.assign(len + 2, 0);
    for (uint32_t v = 0; v < N; ++v) base[__builtin_popcount(v) + 1]++;
    for (int c = 1; c <= len + 1; ++c) base[c] += base[c - 1];
    vals.assign(N, 0);
    std::vector<int> fill(base.begin(), base.end() - 1);
    for (uint32_t v = 0; v < N; ++v) vals[fill[__builtin_popcount(v)]++] = v;
  };
  std::vector<uint32_t> lov, hiv;
  std::vector<int> lob, hib;
  sorted(q, lov, lob);
  sorted(Lh, hiv, hib);
  const uint32_t NL = 1u << q, NH = 1u << Lh;
  std::vector<double> Elo_v(NL), Ehi_v(NH);
  std::vector<int> ndl(NL), ndh(NH);
  for (uint32_t v = 0; v < NL; ++v) Elo_v[v] = half(0, q, v, &ndl[v]);
  for (uint32_t v = 0; v < NH; ++v) Ehi_v[v] = half(q, Lh, v, &ndh[v]);
  std::vector<uint32_t> lo_info(NL), hi_info(NH), hoff(NH, 0);
  std::vector<double> lo_E(NL), hi_E(NH);
  for (uint32_t i = 0; i < NL; ++i) {
    lo_info[i] = lov[i] | ((uint32_t)ndl[lov[i]] << 24);
    lo_E[i] = Elo_v[lov[i]];
  }
  // first row of the block of hi (colex rank contribution of its up spins,
  // which come after the kl up spins of the low half)
  auto block_off = [&](uint32_t v, int kl) {
    int64_t off = 0;
    int j = 0;
    for (int p = 0; p < Lh; ++p)
      if ((v >> p) & 1u) {
        off += Cb(q + p, kl + j + 1);
        ++j;
      }
    return off;
  };
  for (uint32_t i = 0; i < NH; ++i) {
    const uint32_t v = hiv[i];
    hi_info[i] = v | ((uint32_t)ndh[v] << 24);
    hi_E[i] = Ehi_v[v];
    const int kl = k - __builtin_popcount(v);
    if (kl >= 0 && kl <= q) hoff[i] = (uint32_t)block_off(v, kl);
  }
  std::vector<SplitTile> tl[2];
  // low pass: blocks in row order (ascending hi).  Middle bond: for even hi
  // the rows with the top low site up (the last C(q-1, kl-1), from
  // u = C(q-1, kl)) move it to site q, landing on the first rows of the block
  // hi | 1 (k_lo - 1); for odd hi the rows with that site down (u < C(q-1, kl))
  // take the up spin from site q, landing at C(q-1, kl+1) + u in the block
  // hi & ~1 (k_lo + 1).
  for (uint32_t v = 0; v < NH; ++v) {
    const int kl = k - __builtin_popcount(v);
    if (kl < 0 || kl > q) continue;
    SplitTile t{};
    t.row0 = (int32_t)block_off(v, kl);
    t.nrows = (int32_t)Cb(q, kl);
    t.code = v | ((uint32_t)ndh[v] << 24);
    t.aux = lob[kl];
    t.E = Ehi_v[v];
    t.msplit = (int32_t)Cb(q - 1, kl);
    t.mbase = 0;
    const uint32_t pv = v ^ 1u;
    const int pkl = k - __builtin_popcount(pv);
    if (pkl >= 0 && pkl <= q) {
      const int64_t prow0 = block_off(pv, pkl);
      t.mbase = (int32_t)((v & 1u) ? prow0 + Cb(q - 1, kl + 1) : prow0 - Cb(q - 1, kl));
    }
    S.maxmid = std::max(S.maxmid, (int)((v & 1u) ? t.msplit : t.nrows - t.msplit));
    tl[PASS_LOW].push_back(t);
  }
  // high pass: one tile per lo configuration, by (up spins, value)
  for (int kl = std::max(0, k - Lh); kl <= std::min(q, k); ++kl) {
    const int kh = k - kl;
    for (int j = 0; j < (int)Cb(q, kl); ++j) {
      const uint32_t v = lov[lob[kl] + j];
      SplitTile t{};
      t.row0 = j;
      t.nrows = (int32_t)Cb(Lh, kh);
      t.code = v | ((uint32_t)ndl[v] << 24);
      t.aux = hib[kh];
      t.E = Elo_v[v];
      tl[PASS_HIGH].push_back(t);
    }
  }
  for (int ps = 0; ps < 2; ++ps) {
    int64_t rows = 0;
    int mr = 0;
    for (const SplitTile& t : tl[ps]) {
      rows += t.nrows;
      mr = std::max(mr, (int)t.nrows);
    }
    if (rows != H.n) fail(MBL_EINTERNAL, "split tables do not cover the sector");
    S.maxrows[ps] = mr;
    S.ntiles[ps] = (int)tl[ps].size();
    // contiguous tile ranges per XCD with about n/8 rows each
    int64_t acc = 0;
    int x = 1;
    S.xcd_first[ps][0] = 0;
    for (int i = 0; i < (int)tl[ps].size() && x < 8; ++i) {
      acc += tl[ps][i].nrows;
      while (x < 8 && acc * 8 >= (int64_t)x * rows) S.xcd_first[ps][x++] = i + 1;
    }
    while (x <= 8) S.xcd_first[ps][x++] = (int)tl[ps].size();
  }
  auto up = [&](DevBuf& d, const void* src, size_t bytes) {
    H.table(d, std::max<size_t>(bytes, 16), s);
    if (bytes) MBL_HIP(hipMemcpyAsync(d.get(), src, bytes, hipMemcpyHostToDevice, s));
  };
  for (int ps = 0; ps < 2; ++ps) up(S.tiles[ps], tl[ps].data(), tl[ps].size() * sizeof(SplitTile));
  up(S.lo_info, lo_info.data(), lo_info.size() * 4);
  up(S.hi_info, hi_info.data(), hi_info.size() * 4);
  up(S.lo_E, lo_E.data(), lo_E.size() * 8);
  up(S.hi_E, hi_E.data(), hi_E.size() * 8);
  up(S.hoff, hoff.data(), hoff.size() * 4);
  up(S.Elo_v, Elo_v.data(), Elo_v.size() * 8);
  up(S.Ehi_v, Ehi_v.data(), Ehi_v.size() * 8);
  // the host vectors are sources of asynchronous copies
  MBL_HIP(hipStreamSynchronize(s));
  S.ok = true;
}

template bool split_apply<double>(const Ham&, double, const double*, int64_t, double*, int64_t,
                                  int, hipStream_t);
template bool split_apply<float>(const Ham&, double, const float*, int64_t, float*, int64_t, int,
                                 hipStream_t);
template bool split_cg_ready<double>(const Ham&, const SplitCg<double>&);
template bool split_cg_ready<float>(const Ham&, const SplitCg<float>&);
template int split_cg_apply<double>(const Ham&, double, int, const SplitCg<double>&, hipStream_t);
template int split_cg_apply<float>(const Ham&, double, int, const SplitCg<float>&, hipStream_t);

}  // namespace mbl
