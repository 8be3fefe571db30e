// z-update passes (eq. (12), Sec. 4's cyclic convolutions) for power-of-two
// transform lengths N = 64 ... 4096, on the fixed-structure engine of
// fft_p2.h (N / 16 threads per transform, 16 values each in registers).
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
#include "fft_p2.h"

namespace segsalsa {

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
  const int row0 = (bid - m * nrb) * rpb;
  const int nb = min(rpb, H - row0);
  lptr<C2<T>> lds = (lptr<C2<T>>)smem;
  // Fold (fold_rows): 16 elements per thread, stored to each row's LDS region
  fold_rows<T, 16>(a, row0, nb, k0, has1,
                   [&](int rr, int c, C2<T> x) { stc(lds + rr * F::REGION + F::pad(c), x); });
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
