// Internal declarations shared by the SegSALSA-STR HIP kernels and the host runtime.
//
// Data layout (device workspace, one image):
//   The image is cut into a grid of ntr x ntc tiles whose heights (widths)
//   differ by at most one row (column).  Inside a tile the th*tw pixels are
//   numbered row-major and grouped in "steps" of 64 consecutive pixels, one
//   pixel per lane of a wavefront.  Per-pixel solver state is stored
//   tile-major so that every wavefront load/store is one contiguous block:
//     phat [tile][step][K][64]          normalised class probabilities
//     dm   [tile][step][K][3][64]       scaled multipliers d1, d3, d4
//     d2   [tile][step][K][L][64][2]    J-split multipliers (h, v interleaved)
//     acc  [tile][K][ER][EC]            per-tile J^T / identity-split partial sums
//                                       over the tile grown by (M, M+1) on each side
//   z and the spectrum are class-planar: z [K][H][W], spec [P][H][W] complex
//   with P = ceil(K/2) (two classes packed as real and imaginary part).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace segsalsa {

constexpr int kWave = 64;
constexpr int kMaxM = 5;
constexpr int kMaxL = (2 * kMaxM + 1) * (2 * kMaxM + 1);
constexpr int kMaxK = 64;
constexpr int kMaxSide = 4096;
constexpr int kFftEptMax = 16;     // most complex elements per thread in one LDS FFT workgroup
constexpr int kFftMaxThreads = 1024;  // FFT workgroup size limit
// FP64 FFT kernels also come built for workgroups of at most 512 threads
// ("narrow"): under the 1024-thread launch bound the FP64 transforms are held
// to 128 VGPRs and spill, under 512 they get 256 (at half the occupancy).
constexpr int kFftNarrowThreads = 512;
constexpr int kMaxRadices = 24;
constexpr int kLdsMax = 160 * 1024;  // LDS bytes per workgroup on gfx950

template <typename T>
struct C2 {
  T x, y;
};

// Pointers held in device-side descriptor tables reach the kernels as generic
// pointers, which the compiler turns into FLAT accesses; FLAT loads count
// against the LDS wait counter too, so every LDS wait would also wait for
// HBM.  Kernels re-declare them in the global address space.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ inline gptr<T> glob(T* p) {
  return (gptr<T>)p;
}

__host__ __device__ inline int wrap_index(int x, int n) {
  int r = x % n;
  return r < 0 ? r + n : r;
}

// Tile grid of one image.  Tile t covers rows [r0(t), r0(t+1)) and columns
// [c0(t), c0(t+1)); ER x EC is the largest grown tile (th + 2M + 1) x (tw + 2M + 1).
struct TileGeom {
  int H, W, M;
  int ntr, ntc;
  int TR, TC;   // largest tile height / width
  int ER, EC;   // TR + 2M + 1, TC + 2M + 1
  int steps;    // ceil(TR * TC / 64): steps reserved per tile
  __host__ __device__ int r0(int t) const { return (int)(((long long)t * H) / ntr); }
  __host__ __device__ int c0(int t) const { return (int)(((long long)t * W) / ntc); }
  __host__ __device__ int th(int t) const { return r0(t + 1) - r0(t); }
  __host__ __device__ int tw(int t) const { return c0(t + 1) - c0(t); }
  // tile row (column) containing image row (column) x
  __host__ __device__ int trow(int x) const { return (int)((((long long)x + 1) * ntr - 1) / H); }
  __host__ __device__ int tcol(int x) const { return (int)((((long long)x + 1) * ntc - 1) / W); }
  __host__ __device__ int ntiles() const { return ntr * ntc; }
};

// Position of pixel (r, c) in the tile layout: (tile, step, lane).
__host__ __device__ inline void tile_pos(const TileGeom& g, int r, int c, int& tile, int& step, int& lane) {
  const int tr = g.trow(r), tc = g.tcol(c);
  const int f = (r - g.r0(tr)) * g.tw(tc) + (c - g.c0(tc));
  tile = tr * g.ntc + tc;
  step = f >> 6;
  lane = f & 63;
}

// The right-hand side at image row (column) x is the sum of the grown-tile
// partial sums at every grown position that maps onto x periodically.  A
// source row r_s scatters to r_s + [-M, M+1], so only tiles holding a source
// row in x - M - 1 .. x + M contribute.  fold_list writes those positions as
// (tile_row << kFoldShift) | e (e = position inside the grown tile) to
// out[0], out[stride], out[2 stride], ... and returns their number, or -1 if
// there are more than kFoldMax.  The lists of all rows (columns) are stored
// structure-of-arrays, [kFoldStride][n] with the count first, so that the
// lanes of a wavefront reading the lists of consecutive columns read
// consecutive words.
constexpr int kFoldMax = 16;
constexpr int kFoldStride = kFoldMax + 1;   // count + entries per row / column
constexpr int kFoldShift = 13;              // e < ER, EC <= kMaxSide + 2 kMaxM + 1 < 2^13
constexpr int kFoldMask = (1 << kFoldShift) - 1;
static_assert(kMaxSide + 2 * kMaxM + 1 <= kFoldMask, "grown tile position must fit the fold encoding");

__host__ __device__ inline int fold_list(const TileGeom& g, int x, bool is_row, int* out, int stride) {
  const int n = is_row ? g.H : g.W;
  const int M = g.M;
  int cnt = 0;
  for (int d = -M - 1; d <= M; ++d) {
    const int xs = wrap_index(x + d, n);
    const int t = is_row ? g.trow(xs) : g.tcol(xs);
    bool seen = false;
    for (int d2 = -M - 1; d2 < d; ++d2) {
      const int xs2 = wrap_index(x + d2, n);
      seen |= ((is_row ? g.trow(xs2) : g.tcol(xs2)) == t);
    }
    if (seen) continue;
    const int o = is_row ? g.r0(t) : g.c0(t);
    const int lim = (is_row ? g.th(t) : g.tw(t)) + 2 * M;
    for (int e = wrap_index(x - o + M, n); e <= lim; e += n) {
      if (cnt >= kFoldMax) return -1;
      if (out) out[(size_t)cnt * stride] = (t << kFoldShift) | e;
      ++cnt;
    }
  }
  return cnt;
}

// Right-hand side of pixel (r, c), classes k0 and k0 + 1 (has1): the sum of
// the grown-tile partial sums acc[tile][K][ER][EC] covering it, from the fold
// lists rl = frow + r ([kFoldStride][H]) and cl = fcol + c ([kFoldStride][W],
// stride W).  A pixel is almost always covered by at most two tiles per
// direction, so the first 2 x 2 entries are gathered with predicated loads
// whose addresses depend only on the lists (a caller unrolling over several
// pixels gets all their list loads, then all their partial-sum loads, in
// flight together); longer lists (tiles narrower than the halo) add the
// remaining entries in a loop.  Terms are added row entry by row entry.
template <typename T>
__device__ __forceinline__ void fold_gather(__attribute__((address_space(1))) const T* acc,
                                            __attribute__((address_space(1))) const int* rl,
                                            __attribute__((address_space(1))) const int* cl, int H, int W,
                                            const TileGeom& g, int K, int k0, bool has1, T& s0, T& s1) {
  const size_t plane = (size_t)g.ER * g.EC;
  const int nr = rl[0], nc = cl[0];
  const int r0e = rl[H], r1e = rl[2 * H], c0e = cl[W], c1e = cl[2 * W];
  auto rbase = [&](int re) {
    return ((size_t)(re >> kFoldShift) * g.ntc * K + k0) * plane + (size_t)(re & kFoldMask) * g.EC;
  };
  auto cbase = [&](int ce) { return (size_t)(ce >> kFoldShift) * K * plane + (ce & kFoldMask); };
  const size_t rb0 = rbase(r0e), rb1 = rbase(r1e), cb0 = cbase(c0e), cb1 = cbase(c1e);
  const bool r1 = nr > 1, c1 = nc > 1;
  s0 = acc[rb0 + cb0];
  s1 = has1 ? acc[rb0 + cb0 + plane] : T(0);
  if (c1) {
    s0 += acc[rb0 + cb1];
    if (has1) s1 += acc[rb0 + cb1 + plane];
  }
  if (r1) {
    s0 += acc[rb1 + cb0];
    if (has1) s1 += acc[rb1 + cb0 + plane];
    if (c1) {
      s0 += acc[rb1 + cb1];
      if (has1) s1 += acc[rb1 + cb1 + plane];
    }
  }
  if (nr > 2 || nc > 2) {
    for (int i = 0; i < nr; ++i) {
      const size_t rbi = rbase(rl[(size_t)(1 + i) * H]);
      for (int j = 0; j < nc; ++j) {
        if (i < 2 && j < 2) continue;
        const size_t off = rbi + cbase(cl[(size_t)(1 + j) * W]);
        s0 += acc[off];
        if (has1) s1 += acc[off + plane];
      }
    }
  }
}

// Fold of kFoldVec<T> = 16 / sizeof(T) adjacent columns c .. c + kFoldVec - 1
// of one row, for tile geometries where every tile column is tw = W / ntc
// wide, tw a multiple of kFoldVec and tw >= 2M + 2 (a column is then covered
// by its own tile and at most one neighbour, and the group lies in one tile
// column).  Column x = c0 + x0 + j of tile column tc sits at grown position
// x0 + j + M of tile tc; at tw + M + x0 + j of tile tc - 1 when x0 + j <= M;
// at x0 + j - tw + M of tile tc + 1 when x0 + j >= tw - M (tile columns
// taken periodically).  Each term of a row entry is one 16-byte load per
// class; components outside a neighbour's range are dropped by selection
// (their loads reach at most kFoldVec - 1 elements before or after a grown
// row, inside the guard bands around the partial sums).  Row entries come
// from the row list as in fold_gather; the sums are exact per component in
// the same order as fold_gather's (row entry by row entry, own tile column
// before the neighbour).
template <typename T>
constexpr int kFoldVec = 16 / (int)sizeof(T);
constexpr size_t kAccGuard = 256;   // bytes of guard band before and after the partial sums

template <typename T>
struct FoldVec {
  typedef T type __attribute__((ext_vector_type(16 / sizeof(T)), aligned(sizeof(T))));
};

template <typename T>
__device__ __forceinline__ void fold_gather_vec(__attribute__((address_space(1))) const T* acc,
                                                __attribute__((address_space(1))) const int* rl, int H, int c,
                                                const TileGeom& g, int K, int k0, bool has1, T* s0, T* s1) {
  constexpr int V = kFoldVec<T>;
  using VT = typename FoldVec<T>::type;
  const size_t plane = (size_t)g.ER * g.EC;
  const int M = g.M, tw = g.TC;
  const int tc = c / tw, x0 = c - tc * tw;
  const bool left = x0 <= M, right = x0 + V - 1 >= tw - M;
  const int tl = tc == 0 ? g.ntc - 1 : tc - 1, tr = tc + 1 == g.ntc ? 0 : tc + 1;
  const long long co = (long long)tc * K * plane + x0 + M;
  const long long cl = (long long)tl * K * plane + tw + M + x0;
  const long long cr = (long long)tr * K * plane + x0 - tw + M;
  const int nr = rl[0];
  auto rbase = [&](int re) {
    return (long long)(((size_t)(re >> kFoldShift) * g.ntc * K + k0) * plane + (size_t)(re & kFoldMask) * g.EC);
  };
  auto ld = [&](long long off) { return *(__attribute__((address_space(1))) const VT*)(acc + off); };
  // terms in column order (the neighbour on the left, the own tile, the
  // neighbour on the right), the first row entry's starting the sum
  auto add = [&](T* s, long long rb, bool first) {
    const VT o = ld(rb + co);
    const VT l = left ? ld(rb + cl) : VT(0);
    const VT r = right ? ld(rb + cr) : VT(0);
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const bool uj = left && x0 + j <= M, vj = right && x0 + j >= tw - M;
      T t;
      if (first) t = uj ? l[j] + o[j] : o[j];
      else t = uj ? (s[j] + l[j]) + o[j] : s[j] + o[j];
      if (vj) t += r[j];
      s[j] = t;
    }
  };
  const long long rb0 = rbase(rl[H]);
  const long long rb1 = nr > 1 ? rbase(rl[2 * H]) : rb0;
#pragma unroll
  for (int j = 0; j < V; ++j) s1[j] = T(0);
  add(s0, rb0, true);
  if (has1) add(s1, rb0 + (long long)plane, true);
  if (nr > 1) {
    add(s0, rb1, false);
    if (has1) add(s1, rb1 + (long long)plane, false);
  }
  for (int i = 2; i < nr; ++i) {
    const long long rbi = rbase(rl[(size_t)(1 + i) * H]);
    add(s0, rbi, false);
    if (has1) add(s1, rbi + (long long)plane, false);
  }
}

// Workgroups of a launch are dealt to the eight XCDs of the chip round-robin
// (workgroup i runs on XCD i mod 8), and each XCD has its own L2.  Kernels
// whose neighbouring work items share cache lines (the halos of adjacent
// tiles, the adjacent column blocks of one row) renumber their workgroups so
// that each XCD gets runs of kXcdRun consecutive work items: in every group
// of 8 kXcdRun workgroups, XCD x takes items x kXcdRun .. x kXcdRun + kXcdRun - 1
// (the last, partial group is split into eight near-equal runs).  Short runs
// keep the XCDs balanced when the work items of a launch differ in cost (the
// images of a batch).
constexpr int kXcds = 8;
constexpr int kXcdRun = 16;
__device__ inline int xcd_block() {
  const int n = gridDim.x, i = blockIdx.x;
  const int G = kXcds * kXcdRun;
  const int g = i / G, full = n / G;
  const int x = i % kXcds;
  if (g < full) return g * G + x * kXcdRun + (i - g * G) / kXcds;
  const int m = n - full * G, base = full * G;   // the partial group
  const int q = m / kXcds, r = m - q * kXcds, j = (i - base) / kXcds;
  return base + x * q + (x < r ? x : r) + j;
}

// Division of small non-negative integers by a divisor known only at run
// time (a transform length, a block width), as one multiply-high instead of
// the long instruction sequence of an integer division: with
// m = ceil(2^32 / d), umulhi(n, m) = floor(n / d) whenever n d < 2^32.
// Every index divided this way is below 2^15 and every divisor below 2^13;
// d = 1 (multiplier 2^32) is taken apart.
struct FastDiv {
  uint32_t d, m;
  __device__ explicit FastDiv(uint32_t dd) : d(dd), m(dd > 1 ? 0xFFFFFFFFu / dd + 1u : 0u) {}
  __device__ uint32_t div(uint32_t n) const { return d == 1 ? n : __umulhi(n, m); }
  __device__ uint32_t mod(uint32_t n) const { return n - div(n) * d; }
};

// Per-pixel arithmetic parameters of one round.
enum PKind : int { kSchatten1 = 1, kSchatten2 = 2, kSchattenInf = 3, kSchattenP = 4 };

// Per-image kernel arguments live in device tables; a launch covers a range
// of images and block b belongs to the last image whose block0 <= b.
template <typename D>
__device__ inline int find_desc(const D* descs, int n, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].block0 <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename T>
struct ProxArgs {
  int block0;                 // first block of this image in the launch
  TileGeom g;
  int K;
  int nw;                     // wavefronts per workgroup
  const T* __restrict__ z;    // [K][H][W]
  const T* __restrict__ phat; // tile layout
  // multipliers of the round's input state (d1, d3, d4 and d2, tile layout)
  // and where the updated ones go: the same arrays for an update in place,
  // another state's for rounds that keep every state (the reverse sweep)
  const T* dm_in;
  const T* d2_in;
  T* dm;
  T* d2;
  T* __restrict__ acc;
  double* __restrict__ res_tile;  // non-null on checked rounds: per-tile sum of (d_new - d_old)^2
  double mu, tau;
  int pkind;
  double pval;                // the Schatten p (used when pkind == kSchattenP)
  int g4s;                    // 1: g4 is the probability-simplex projection
  T c[kMaxL];
};

// One 1-D DFT length.  Mixed-radix Stockham over the factors in rad[], or,
// for lengths with a large prime factor (blu = 1), Bluestein's chirp
// transform: a length-M cyclic convolution (M a power of two >= 2N - 1)
// computed with the power-of-two radices in mrad[].
struct FftPlanDev {
  int N;
  int nst;
  int rad[kMaxRadices];
  int blu;
  int M;
  int mnst;
  int mrad[kMaxRadices];
};

// Tables of one DFT length (device memory).
template <typename T>
struct FftTab {
  const C2<T>* tw;     // N twiddles exp(-2 pi i t / N) (Stockham path)
  const C2<T>* chirp;  // N values exp(-i pi n^2 / N) (Bluestein)
  const C2<T>* bf;     // M values: DFT_M of the kernel exp(+i pi m^2 / N) wrapped cyclically (Bluestein)
  const C2<T>* twM;    // M twiddles exp(-2 pi i t / M) (Bluestein)
};

template <typename T>
struct RowFwdArgs {
  int block0;
  TileGeom g;
  int K, P;
  int rows_per_block;
  int vfold;                    // 1: tile columns allow fold_gather_vec
  const T* __restrict__ acc;    // per-tile partial sums
  const int* __restrict__ frow; // [kFoldStride][H] fold lists of rows
  const int* __restrict__ fcol; // [kFoldStride][W] fold lists of columns
  C2<T>* __restrict__ spec;     // [P][H][W]
  FftTab<T> tab;                // row-length tables
  FftPlanDev plan;
};

template <typename T>
struct ColArgs {
  int block0;
  int H, W, P;
  int cols_per_block;
  C2<T>* __restrict__ spec;
  FftTab<T> tab;                  // column-length tables
  const double* __restrict__ sx;  // 4 sin^2(pi kx / W)
  const double* __restrict__ sy;  // 4 sin^2(pi ky / H)
  double wsum;                    // sum_j c_j^2
  double scale;                   // 1 / (H W)
  FftPlanDev plan;
};

template <typename T>
struct RowInvArgs {
  int block0;
  int H, W, K, P;
  int rows_per_block;
  const C2<T>* __restrict__ spec;
  T* __restrict__ z;
  FftTab<T> tab;
  FftPlanDev plan;
};

}  // namespace segsalsa
