// z-update passes (eq. (12), Sec. 4's cyclic convolutions) for power-of-two
// transform lengths N = 64 ... 4096, with the whole transform structure
// fixed at compile time.
//
// Each transform of N points is handled by N / 16 threads that each hold 16
// complex values in registers: thread t holds x[t + (N/16) q], q = 0 .. 15.
// The transform is a Stockham autosort FFT of radix-16 stages and one last
// stage of radix N / 16^s: in every stage a thread runs 16 / R butterflies of
// radix R, butterfly j = t + (N/16) u taking the inputs x[j + r N / R]
// = x[t + (N/16)(u + r 16/R)], so the thread's inputs are always its own 16
// values.  Between stages the outputs go through LDS (with one pad word every
// 16 elements against bank conflicts); the last stage's outputs X[j + r N/R]
// are again X[t + (N/16) q] and stay in registers.  All index arithmetic is
// with compile-time powers of two, so it is shifts and masks, and a stage
// costs one LDS write and one LDS read per element.
//
// Kernels (same descriptors as the general kernels of fft_kernels.hip):
//   rows_fwd: fold of the grown-tile partial sums straight into registers,
//             class pairs packed as complex, forward DFT of each row
//   cols:     forward DFT of each column, division by the symbol of G^T G
//             (and by H W), inverse DFT, without leaving registers between
//             the two transforms
//   rows_inv: inverse DFT of each row, unpacked into the two class planes
#include "segsalsa_internal.h"
#include "segsalsa_kernels.h"
#include "fft_math.h"

namespace segsalsa {

// DFT of 16 values as 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2, so that
// w^(nk) = (w^4)^(n1 k1) w^(n2 k1) (w^4)^(n2 k2) with w = exp(sg 2 pi i / 16):
// radix-4 over n1, the twiddles w^(n2 k1), radix-4 over n2.
template <typename T>
__device__ __forceinline__ void bfly16(C2<T>* v, T sg) {
  const T c1 = T(0.92387953251128675613);  // cos(pi / 8)
  const T s1 = T(0.38268343236508977173);  // sin(pi / 8)
  const T r2 = T(0.70710678118654752440);  // cos(pi / 4)
  C2<T> A[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    C2<T> x[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
    Bfly<T, 4>::run(x, sg);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) A[n2][k1] = x[k1];
  }
  // w^m for m = n2 k1 in {1, 2, 3, 4, 6, 9}: (cos(2 pi m / 16), sg sin(2 pi m / 16))
  auto tw = [&](C2<T> a, T wr, T wi) { return C2<T>{a.x * wr - a.y * wi, a.x * wi + a.y * wr}; };
  A[1][1] = tw(A[1][1], c1, sg * s1);
  A[1][2] = tw(A[1][2], r2, sg * r2);
  A[1][3] = tw(A[1][3], s1, sg * c1);
  A[2][1] = tw(A[2][1], r2, sg * r2);
  A[2][2] = cmuli(A[2][2], sg);
  A[2][3] = tw(A[2][3], -r2, sg * r2);
  A[3][1] = tw(A[3][1], s1, sg * c1);
  A[3][2] = tw(A[3][2], -r2, sg * r2);
  A[3][3] = tw(A[3][3], -c1, -sg * s1);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    C2<T> x[4] = {A[0][k1], A[1][k1], A[2][k1], A[3][k1]};
    Bfly<T, 4>::run(x, sg);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = x[k2];
  }
}

template <typename T, int R>
__device__ __forceinline__ void bfly_p2(C2<T>* v, T sg) {
  if constexpr (R == 16) bfly16<T>(v, sg);
  else Bfly<T, R>::run(v, sg);
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

template <typename T, int N>
struct P2Fft {
  static_assert(N >= 64 && N <= 4096 && (N & (N - 1)) == 0, "power-of-two length 64 .. 4096");
  static constexpr int LG = ilog2(N);
  static constexpr int TPT = N / 16;                          // threads per transform
  static constexpr int NST = (LG + 3) / 4;                    // stages
  static constexpr int LAST = LG % 4 == 0 ? 16 : (1 << (LG % 4));
  static constexpr int REGION = N + N / 16 + 1;               // LDS elements per transform
  static constexpr int radix(int s) { return s < NST - 1 ? 16 : LAST; }
  static constexpr int span(int s) { return s == 0 ? 1 : span(s - 1) * radix(s - 1); }   // Ns of stage s
  __device__ static int pad(int i) { return i + (i >> 4); }

  template <int S>
  __device__ __forceinline__ static void stage(C2<T> (&v)[16], lptr<C2<T>> buf, int t, gptr<const C2<T>> tw,
                                               bool inv) {
    constexpr int R = radix(S), NS = span(S), U = 16 / R, STRIDE = N / (NS * R);
    constexpr bool last = S == NST - 1;
    if constexpr (S > 0) {   // inputs: the previous stage's outputs in LDS
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = ldc(buf + pad(t + TPT * q));
      if constexpr (!last) __syncthreads();   // every read done before this stage overwrites the region
    }
    const T sg = inv ? T(1) : T(-1);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = t + TPT * u;
      const int k = j & (NS - 1);
      C2<T> x[R];
#pragma unroll
      for (int r = 0; r < R; ++r) x[r] = v[u + r * U];
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) x[r] = twmul(x[r], ldc(tw + r * k * STRIDE), inv);   // r k STRIDE < N
      }
      bfly_p2<T, R>(x, sg);
      if constexpr (last) {   // output j + r NS = t + TPT (u + r U): the thread's own slots
#pragma unroll
        for (int r = 0; r < R; ++r) v[u + r * U] = x[r];
      } else {
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) stc(buf + pad(base + r * NS), x[r]);
      }
    }
  }

  // Unnormalised DFT of one transform, inv = false: exp(-2 pi i ...), true:
  // exp(+2 pi i ...).  v[q] = x[t + TPT q] on entry, X[t + TPT q] on exit.
  // buf: the transform's LDS region; tw: exp(-2 pi i m / N), m < N.  Every
  // thread of the workgroup calls it at the same time (it holds barriers).
  __device__ __forceinline__ static void run(C2<T> (&v)[16], lptr<C2<T>> buf, int t, gptr<const C2<T>> tw,
                                             bool inv) {
    stage<0>(v, buf, t, tw, inv);
    if constexpr (NST > 1) stage<1>(v, buf, t, tw, inv);
    if constexpr (NST > 2) stage<2>(v, buf, t, tw, inv);
    static_assert(NST <= 3, "at most three stages for N <= 4096");
  }
};

template <typename T>
constexpr int p2_max_threads() {
  return sizeof(T) == 8 ? kFftNarrowThreads : kFftMaxThreads;
}

template <typename T, int N>
__global__ void __launch_bounds__(p2_max_threads<T>()) fft_rows_fwd_p2_kernel(const RowFwdArgs<T>* __restrict__ descs,
                                                                           int ndesc) {
  using F = P2Fft<T, N>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int blk = xcd_block();   // consecutive rows (neighbouring grown-tile rows) on one XCD
  const RowFwdArgs<T>& a = descs[find_desc(descs, ndesc, blk)];
  const int bid = blk - a.block0;
  const int H = a.g.H;
  const int rpb = a.rows_per_block;
  const int nrb = (H + rpb - 1) / rpb;
  const int m = bid / nrb;
  const int tb = threadIdx.x / F::TPT, t = threadIdx.x & (F::TPT - 1);
  const int r = (bid - m * nrb) * rpb + tb;
  const bool active = r < H;
  const int k0 = 2 * m, k1 = 2 * m + 1;
  const bool has1 = k1 < a.K;
  const size_t plane = (size_t)a.g.ER * a.g.EC;
  const gptr<const T> acc = glob(a.acc);
  const gptr<const int> frow = glob(a.frow), fcol = glob(a.fcol);
  const int row0 = (bid - m * nrb) * rpb;
  const int nb = min(rpb, H - row0);
  lptr<C2<T>> lds = (lptr<C2<T>>)smem;
  // Fold: right-hand side = sum of the grown-tile partial sums covering
  // (r, c), from the fold lists [kFoldStride][n] (count, entries), into each
  // row's LDS region.  The workgroup's nb * N elements are 16 per thread;
  // the loop is unrolled and each list's first two entries are read with its
  // count, so the list and data loads of a thread's elements are in flight
  // together (most pixels have one or two entries per direction).
#pragma unroll
  for (int it = 0; it < 16; ++it) {
    const int idx = threadIdx.x + it * blockDim.x;
    const int rr = idx >> F::LG, c = idx & (N - 1);
    if (rr < nb) {
      const gptr<const int> rl = frow + (row0 + rr);
      const gptr<const int> cl = fcol + c;
      const int nr = rl[0], nc = cl[0];
      const int r0e = rl[H], r1e = rl[2 * H], c0e = cl[N], c1e = cl[2 * N];
      T s0 = T(0), s1 = T(0);
      for (int i = 0; i < nr; ++i) {
        const int ri = i == 0 ? r0e : (i == 1 ? r1e : rl[(size_t)(1 + i) * H]);
        const int tr = ri >> kFoldShift, er = ri & kFoldMask;
        for (int j = 0; j < nc; ++j) {
          const int cj = j == 0 ? c0e : (j == 1 ? c1e : cl[(size_t)(1 + j) * N]);
          const size_t tile = (size_t)tr * a.g.ntc + (cj >> kFoldShift);
          const size_t off = ((tile * a.K + k0) * plane) + (size_t)er * a.g.EC + (cj & kFoldMask);
          s0 += acc[off];
          if (has1) s1 += acc[off + plane];
        }
      }
      stc(lds + rr * F::REGION + F::pad(c), C2<T>{s0, s1});
    }
  }
  __syncthreads();
  C2<T> v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = ldc(lds + tb * F::REGION + F::pad(t + F::TPT * q));
  __syncthreads();   // every element read before the first stage overwrites the regions
  F::run(v, (lptr<C2<T>>)smem + tb * F::REGION, t, glob(a.tab.tw), false);
  if (active) {
    const gptr<C2<T>> out = glob(a.spec) + ((size_t)m * H + r) * N + t;
#pragma unroll
    for (int q = 0; q < 16; ++q) stc(out + F::TPT * q, v[q]);
  }
}

template <typename T, int N>
__global__ void __launch_bounds__(p2_max_threads<T>()) fft_cols_p2_kernel(const ColArgs<T>* __restrict__ descs,
                                                                       int ndesc) {
  using F = P2Fft<T, N>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int blk = xcd_block();   // adjacent column blocks (shared cache lines) on one XCD
  const ColArgs<T>& a = descs[find_desc(descs, ndesc, blk)];
  const int bid = blk - a.block0;
  const int W = a.W;
  const int cpb = a.cols_per_block;
  const int ncb = (W + cpb - 1) / cpb;
  const int m = bid / ncb;
  // lanes take consecutive columns first, so that a load or store of one
  // element slot touches cpb adjacent columns of several rows
  const FastDiv fc(cpb);
  const int t = (int)fc.div(threadIdx.x), j = threadIdx.x - t * cpb;
  const int x = (bid - m * ncb) * cpb + j;
  const bool active = x < W;
  const gptr<C2<T>> sp = glob(a.spec) + (size_t)m * N * W + x;
  C2<T> v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = active ? ldc(sp + (size_t)(t + F::TPT * q) * W) : C2<T>{T(0), T(0)};
  const lptr<C2<T>> buf = (lptr<C2<T>>)smem + j * F::REGION;
  const gptr<const C2<T>> tw = glob(a.tab.tw);
  F::run(v, buf, t, tw, false);
  // division by the symbol 3 + Wsum (4 sin^2(pi kx / W) + 4 sin^2(pi ky / H)) and by H W
  const gptr<const double> sx = glob(a.sx), sy = glob(a.sy);
  const T sxx = active ? T(sx[x]) : T(0);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const T inv = T(a.scale) / (T(3) + T(a.wsum) * (sxx + T(sy[t + F::TPT * q])));
    v[q] = cscale(v[q], inv);
  }
  __syncthreads();   // the forward transform's last reads are done before the inverse writes
  F::run(v, buf, t, tw, true);
  if (active) {
#pragma unroll
    for (int q = 0; q < 16; ++q) stc(sp + (size_t)(t + F::TPT * q) * W, v[q]);
  }
}

template <typename T, int N>
__global__ void __launch_bounds__(p2_max_threads<T>()) fft_rows_inv_p2_kernel(const RowInvArgs<T>* __restrict__ descs,
                                                                           int ndesc) {
  using F = P2Fft<T, N>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int blk = xcd_block();
  const RowInvArgs<T>& a = descs[find_desc(descs, ndesc, blk)];
  const int bid = blk - a.block0;
  const int H = a.H;
  const int rpb = a.rows_per_block;
  const int nrb = (H + rpb - 1) / rpb;
  const int m = bid / nrb;
  const int tb = threadIdx.x / F::TPT, t = threadIdx.x & (F::TPT - 1);
  const int r = (bid - m * nrb) * rpb + tb;
  const bool active = r < H;
  const gptr<const C2<T>> in = glob(a.spec) + ((size_t)m * H + r) * N + t;
  C2<T> v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = active ? ldc(in + F::TPT * q) : C2<T>{T(0), T(0)};
  F::run(v, (lptr<C2<T>>)smem + tb * F::REGION, t, glob(a.tab.tw), true);
  if (active) {
    const int k0 = 2 * m, k1 = 2 * m + 1;
    const gptr<T> z0 = glob(a.z) + ((size_t)k0 * H + r) * N + t;
    const gptr<T> z1 = glob(a.z) + ((size_t)k1 * H + r) * N + t;
    const bool has1 = k1 < a.K;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      z0[F::TPT * q] = v[q].x;
      if (has1) z1[F::TPT * q] = v[q].y;
    }
  }
}

template <auto FN, typename A>
static hipError_t launch_p2(const A* descs, int ndesc, int blocks, int threads, size_t lds, hipStream_t st) {
  static bool lds_set = false;  // idempotent, so a racing second call is harmless
  if (!lds_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(FN),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kLdsMax);
    if (e != hipSuccess) return e;
    lds_set = true;
  }
  hipLaunchKernelGGL(FN, dim3(blocks), dim3(threads), lds, st, descs, ndesc);
  return hipGetLastError();
}

#define SEG_P2_LAUNCHER(NAME, ARGS, KERNEL)                                                                         \
  template <typename T>                                                                                           \
  static hipError_t NAME##_t(const ARGS<T>* d, int n, int blocks, int N, int threads, size_t lds, hipStream_t st) { \
    switch (N) {                                                                                                  \
      case 64: return launch_p2<KERNEL<T, 64>>(d, n, blocks, threads, lds, st);                                   \
      case 128: return launch_p2<KERNEL<T, 128>>(d, n, blocks, threads, lds, st);                                 \
      case 256: return launch_p2<KERNEL<T, 256>>(d, n, blocks, threads, lds, st);                                 \
      case 512: return launch_p2<KERNEL<T, 512>>(d, n, blocks, threads, lds, st);                                 \
      case 1024: return launch_p2<KERNEL<T, 1024>>(d, n, blocks, threads, lds, st);                               \
      case 2048: return launch_p2<KERNEL<T, 2048>>(d, n, blocks, threads, lds, st);                               \
      case 4096: return launch_p2<KERNEL<T, 4096>>(d, n, blocks, threads, lds, st);                               \
      default: return hipErrorInvalidValue;                                                                       \
    }                                                                                                             \
  }                                                                                                               \
  hipError_t NAME(const ARGS<float>* d, int n, int blocks, int N, int threads, size_t lds, hipStream_t st) {       \
    return NAME##_t<float>(d, n, blocks, N, threads, lds, st);                                                    \
  }                                                                                                               \
  hipError_t NAME(const ARGS<double>* d, int n, int blocks, int N, int threads, size_t lds, hipStream_t st) {      \
    return NAME##_t<double>(d, n, blocks, N, threads, lds, st);                                                   \
  }

SEG_P2_LAUNCHER(launch_rows_fwd_p2, RowFwdArgs, fft_rows_fwd_p2_kernel)
SEG_P2_LAUNCHER(launch_cols_p2, ColArgs, fft_cols_p2_kernel)
SEG_P2_LAUNCHER(launch_rows_inv_p2, RowInvArgs, fft_rows_inv_p2_kernel)
#undef SEG_P2_LAUNCHER

}  // namespace segsalsa
