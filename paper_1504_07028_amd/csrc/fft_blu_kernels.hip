// z-update passes (eq. (12), Sec. 4's cyclic convolutions) for sides with a
// prime factor above the direct stages' range, by Bluestein's chirp
// transform with its two length-M convolution FFTs (M a power of two,
// 2N - 1 <= M <= 4096) on the fixed-structure engine of fft_p2.h.
//
// A length-N DFT X_k = c_k sum_n (x_n c_n) d_(k-n), c_n = exp(-i pi n^2 / N),
// d = conj(c), is the cyclic convolution of x c (zero-padded to M) with the
// kernel d wrapped onto M points: IDFT_M(DFT_M(x c) DFT_M(d)) / M, read at
// k < N and multiplied by c_k.  DFT_M(d) is the precomputed table bf; the
// inverse DFT takes conj(c) and conj(bf) read at -m.  Each transform's M / 16
// threads hold its values in registers from the chirp in to the chirp out;
// thread t holds the indices t + (M/16) q, so the N inputs and outputs are
// the same register slots and the column pass runs forward transform,
// symbol division and inverse transform without leaving registers.
//
// Kernels (same descriptors as the general kernels of fft_kernels.hip):
//   rows_fwd: fold of the grown-tile partial sums into LDS, class pairs
//             packed as complex, forward DFT of each row
//   cols:     forward DFT of each column, division by the symbol of G^T G
//             (and by H W), inverse DFT
//   rows_inv: inverse DFT of each row, unpacked into the two class planes
#include "segsalsa_internal.h"
#include "segsalsa_kernels.h"
#include "fft_math.h"
#include "fft_p2.h"

namespace segsalsa {

// Length-n DFT (inv = false: exp(-2 pi i ...), true: exp(+2 pi i ...)) by
// Bluestein over MM points.  On entry v[q] = x[t + (MM/16) q] for indices
// below n (the others are ignored); on exit v[q] = X[t + (MM/16) q] for
// indices below n.  buf is the transform's LDS region.  Starts with a
// barrier (the region may still be read by a previous pass); every thread
// of the workgroup calls it at the same time.
template <typename T, int MM>
__device__ __forceinline__ void blu_dft(C2<T> (&v)[16], int n, lptr<C2<T>> buf, int t, const FftTab<T>& tab,
                                        bool inv) {
  using F = P2Fft<T, MM>;
  const gptr<const C2<T>> ch = glob(tab.chirp), bf = glob(tab.bf), tw = glob(tab.twM);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = t + F::TPT * q;
    if (idx < n) {
      C2<T> c = ldc(ch + idx);
      if (inv) c.y = -c.y;
      v[q] = cmul(v[q], c);
    } else {
      v[q] = C2<T>{T(0), T(0)};
    }
  }
  __syncthreads();
  F::run(v, buf, t, tw, false);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = t + F::TPT * q;
    C2<T> w;
    if (inv) {  // DFT of conj(d) is conj(DFT(d)) read at -m
      w = ldc(bf + ((MM - idx) & (MM - 1)));
      w.y = -w.y;
    } else {
      w = ldc(bf + idx);
    }
    v[q] = cmul(v[q], w);
  }
  __syncthreads();   // the forward transform's last reads are done before the inverse writes
  F::run(v, buf, t, tw, true);
  const T invM = T(1) / T(MM);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = t + F::TPT * q;
    if (idx < n) {
      C2<T> c = ldc(ch + idx);
      if (inv) c.y = -c.y;
      v[q] = cscale(cmul(v[q], c), invM);
    }
  }
}

template <typename T, int MM>
__global__ void __launch_bounds__(p2_max_threads<T>()) fft_rows_fwd_blu_kernel(const RowFwdArgs<T>* __restrict__ descs,
                                                                            int ndesc) {
  using F = P2Fft<T, MM>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int blk = xcd_block();   // consecutive rows (neighbouring grown-tile rows) on one XCD
  const RowFwdArgs<T>& a = descs[find_desc(descs, ndesc, blk)];
  const int bid = blk - a.block0;
  const int H = a.g.H, W = a.g.W;
  const int rpb = a.rows_per_block;
  const int nrb = (H + rpb - 1) / rpb;
  const int m = bid / nrb;
  const int tb = threadIdx.x / F::TPT, t = threadIdx.x & (F::TPT - 1);
  const int row0 = (bid - m * nrb) * rpb;
  const int r = row0 + tb;
  const bool active = r < H;
  const int nb = min(rpb, H - row0);
  const int k0 = 2 * m, k1 = 2 * m + 1;
  const bool has1 = k1 < a.K;
  lptr<C2<T>> lds = (lptr<C2<T>>)smem;
  // Fold (fold_rows): the workgroup's nb * W elements are at most 8 per
  // thread (W <= MM / 2), stored to each row's LDS region
  fold_rows<T, 8>(a, row0, nb, k0, has1, [&](int rr, int c, C2<T> x) { stc(lds + rr * F::REGION + F::pad(c), x); });
  __syncthreads();
  C2<T> v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = t + F::TPT * q;
    v[q] = idx < W ? ldc(lds + tb * F::REGION + F::pad(idx)) : C2<T>{T(0), T(0)};
  }
  blu_dft<T, MM>(v, W, lds + tb * F::REGION, t, a.tab, false);
  if (active) {
    const gptr<C2<T>> out = glob(a.spec) + ((size_t)m * H + r) * W;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int idx = t + F::TPT * q;
      if (idx < W) stc(out + idx, v[q]);
    }
  }
}

// at most kFftNarrowThreads threads: the four transforms and the symbol keep
// more values live than the 128 registers of a 1024-thread workgroup hold
template <typename T, int MM>
__global__ void __launch_bounds__(kFftNarrowThreads) fft_cols_blu_kernel(const ColArgs<T>* __restrict__ descs,
                                                                      int ndesc) {
  using F = P2Fft<T, MM>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int blk = xcd_block();   // adjacent column blocks (shared cache lines) on one XCD
  const ColArgs<T>& a = descs[find_desc(descs, ndesc, blk)];
  const int bid = blk - a.block0;
  const int H = a.H, W = a.W;
  const int cpb = a.cols_per_block;
  const int ncb = (W + cpb - 1) / cpb;
  const int m = bid / ncb;
  // lanes take consecutive columns first, so that a load or store of one
  // element slot touches cpb adjacent columns of several rows
  const FastDiv fc(cpb);
  const int t = (int)fc.div(threadIdx.x), j = threadIdx.x - t * cpb;
  const int x = (bid - m * ncb) * cpb + j;
  const bool active = x < W;
  const gptr<C2<T>> sp = glob(a.spec) + (size_t)m * H * W + x;
  C2<T> v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = t + F::TPT * q;
    v[q] = active && idx < H ? ldc(sp + (size_t)idx * W) : C2<T>{T(0), T(0)};
  }
  const lptr<C2<T>> buf = (lptr<C2<T>>)smem + j * F::REGION;
  blu_dft<T, MM>(v, H, buf, t, a.tab, false);
  // division by the symbol 3 + Wsum (4 sin^2(pi kx / W) + 4 sin^2(pi ky / H)) and by H W
  const gptr<const double> sx = glob(a.sx), sy = glob(a.sy);
  const T sxx = active ? T(sx[x]) : T(0);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = t + F::TPT * q;
    if (idx < H) v[q] = cscale(v[q], T(a.scale) / (T(3) + T(a.wsum) * (sxx + T(sy[idx]))));
  }
  blu_dft<T, MM>(v, H, buf, t, a.tab, true);
  if (active) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int idx = t + F::TPT * q;
      if (idx < H) stc(sp + (size_t)idx * W, v[q]);
    }
  }
}

template <typename T, int MM>
__global__ void __launch_bounds__(p2_max_threads<T>()) fft_rows_inv_blu_kernel(const RowInvArgs<T>* __restrict__ descs,
                                                                            int ndesc) {
  using F = P2Fft<T, MM>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int blk = xcd_block();
  const RowInvArgs<T>& a = descs[find_desc(descs, ndesc, blk)];
  const int bid = blk - a.block0;
  const int H = a.H, W = a.W;
  const int rpb = a.rows_per_block;
  const int nrb = (H + rpb - 1) / rpb;
  const int m = bid / nrb;
  const int tb = threadIdx.x / F::TPT, t = threadIdx.x & (F::TPT - 1);
  const int r = (bid - m * nrb) * rpb + tb;
  const bool active = r < H;
  const gptr<const C2<T>> in = glob(a.spec) + ((size_t)m * H + r) * W;
  C2<T> v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = t + F::TPT * q;
    v[q] = active && idx < W ? ldc(in + idx) : C2<T>{T(0), T(0)};
  }
  blu_dft<T, MM>(v, W, (lptr<C2<T>>)smem + tb * F::REGION, t, a.tab, true);
  if (active) {
    const int k0 = 2 * m, k1 = 2 * m + 1;
    const gptr<T> z0 = glob(a.z) + ((size_t)k0 * H + r) * W;
    const gptr<T> z1 = glob(a.z) + ((size_t)k1 * H + r) * W;
    const bool has1 = k1 < a.K;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int idx = t + F::TPT * q;
      if (idx < W) {
        z0[idx] = v[q].x;
        if (has1) z1[idx] = v[q].y;
      }
    }
  }
}

template <auto FN, typename A>
static hipError_t launch_blu(const A* descs, int ndesc, int blocks, int threads, size_t lds, hipStream_t st) {
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

// MM: the Bluestein length, 64 .. 4096 (256 .. 4096 for the sides 101 .. 2048
// whose prime factors above 100 take Bluestein by default)
#define SEG_BLU_LAUNCHER(NAME, ARGS, KERNEL)                                                                         \
  template <typename T>                                                                                            \
  static hipError_t NAME##_t(const ARGS<T>* d, int n, int blocks, int MM, int threads, size_t lds, hipStream_t st) { \
    switch (MM) {                                                                                                  \
      case 64: return launch_blu<KERNEL<T, 64>>(d, n, blocks, threads, lds, st);                                   \
      case 128: return launch_blu<KERNEL<T, 128>>(d, n, blocks, threads, lds, st);                                 \
      case 256: return launch_blu<KERNEL<T, 256>>(d, n, blocks, threads, lds, st);                                 \
      case 512: return launch_blu<KERNEL<T, 512>>(d, n, blocks, threads, lds, st);                                 \
      case 1024: return launch_blu<KERNEL<T, 1024>>(d, n, blocks, threads, lds, st);                               \
      case 2048: return launch_blu<KERNEL<T, 2048>>(d, n, blocks, threads, lds, st);                               \
      case 4096: return launch_blu<KERNEL<T, 4096>>(d, n, blocks, threads, lds, st);                               \
      default: return hipErrorInvalidValue;                                                                        \
    }                                                                                                              \
  }                                                                                                                \
  hipError_t NAME(const ARGS<float>* d, int n, int blocks, int MM, int threads, size_t lds, hipStream_t st) {       \
    return NAME##_t<float>(d, n, blocks, MM, threads, lds, st);                                                    \
  }                                                                                                                \
  hipError_t NAME(const ARGS<double>* d, int n, int blocks, int MM, int threads, size_t lds, hipStream_t st) {      \
    return NAME##_t<double>(d, n, blocks, MM, threads, lds, st);                                                   \
  }

SEG_BLU_LAUNCHER(launch_rows_fwd_blu, RowFwdArgs, fft_rows_fwd_blu_kernel)
SEG_BLU_LAUNCHER(launch_cols_blu, ColArgs, fft_cols_blu_kernel)
SEG_BLU_LAUNCHER(launch_rows_inv_blu, RowInvArgs, fft_rows_inv_blu_kernel)
#undef SEG_BLU_LAUNCHER

}  // namespace segsalsa
