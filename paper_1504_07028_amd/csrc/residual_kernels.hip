// Convergence diagnostics of SegSALSA-STR: dual residual, objective of
// eq. (7) at the simplex projection of z, and their fixed-order reductions.
//
// Primal residual (computed inside the prox kernel): ||G z - u||_F, which by
// the multiplier update of eq. (14) equals ||d_new - d_old||_F.
// Dual residual: mu ||G (z_new - z_old)||_F with
//   ||G x||^2 = 3 ||x||^2 + ||J x||^2 = 3 ||x||^2 + Wsum (||D_h x||^2 + ||D_v x||^2),
// a local stencil because the periodic shifts P_j are orthogonal.
// All sums are accumulated in FP64 and reduced in a fixed order.
#include <algorithm>

#include "segsalsa_internal.h"
#include "segsalsa_kernels.h"

namespace segsalsa {

// Sum of v over the workgroup, valid in thread 0 (fixed order).
__device__ inline double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  __syncthreads();
  return t;
}

template <typename T>
__global__ void __launch_bounds__(256) copy_kernel(const T* __restrict__ src, T* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

template <typename T>
__global__ void __launch_bounds__(256) dual_res_kernel(const DiagArgs<T> a) {
  __shared__ double sh[4];
  const int H = a.g.H, W = a.g.W;
  const size_t n = (size_t)H * W;
  const size_t total = n * a.K;
  double acc = 0.0;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const size_t k = e / n, i = e - k * n;
    const int r = (int)(i / W), c = (int)(i - (size_t)r * W);
    const T* zk = a.z + k * n;
    const T* pk = a.zprev + k * n;
    const size_t ir = (size_t)r * W + (c + 1 == W ? 0 : c + 1);
    const size_t id = (size_t)(r + 1 == H ? 0 : r + 1) * W + c;
    const double d0 = (double)zk[i] - (double)pk[i];
    const double dr = (double)zk[ir] - (double)pk[ir];
    const double dd = (double)zk[id] - (double)pk[id];
    acc += 3.0 * d0 * d0 + a.wsum * ((dr - d0) * (dr - d0) + (dd - d0) * (dd - d0));
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) a.partial[blockIdx.x] = t;
}

// Euclidean projection of every z_i onto the probability simplex (exact,
// iterative removal of the components at or below the threshold).
template <typename T>
__global__ void __launch_bounds__(256) simplex_kernel(const DiagArgs<T> a) {
  const size_t n = (size_t)a.g.H * a.g.W;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int K = a.K;
  double theta = 0.0;
  unsigned long long active = K >= 64 ? ~0ull : ((1ull << K) - 1ull);
  for (int it = 0; it <= K; ++it) {
    double s = 0.0;
    int cnt = 0;
    for (int k = 0; k < K; ++k)
      if (active >> k & 1ull) {
        s += (double)a.z[(size_t)k * n + i];
        ++cnt;
      }
    theta = (s - 1.0) / cnt;
    unsigned long long next = 0;
    for (int k = 0; k < K; ++k)
      if ((active >> k & 1ull) && (double)a.z[(size_t)k * n + i] > theta) next |= 1ull << k;
    if (next == active || next == 0) break;
    active = next;
  }
  for (int k = 0; k < K; ++k) {
    const double v = (double)a.z[(size_t)k * n + i] - theta;
    a.zprev[(size_t)k * n + i] = T(v > 0.0 ? v : 0.0);
  }
}

// Per pixel: -ln(p_hat^T zp_i) + lambda ||[J zp]_i||_{S_p} with zp the projected field (in a.zprev).
template <typename T>
__global__ void __launch_bounds__(256) objective_kernel(const DiagArgs<T> a) {
  __shared__ double sh[4];
  const int H = a.g.H, W = a.g.W, K = a.K, M = a.g.M;
  const size_t n = (size_t)H * W;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double val = 0.0;
  if (i < n) {
    const int r = (int)(i / W), c = (int)(i - (size_t)r * W);
    const int tr = a.g.trow(r), tc = a.g.tcol(c);
    const int f = (r - a.g.r0(tr)) * a.g.tw(tc) + (c - a.g.c0(tc));
    const size_t sb = (((size_t)tr * a.g.ntc + tc) * a.g.steps + (f >> 6)) * K;
    double dot = 0.0;
    for (int k = 0; k < K; ++k) dot += (double)a.phat[(sb + k) * 64 + (f & 63)] * (double)a.zprev[(size_t)k * n + i];
    double A = 0.0, B = 0.0, C = 0.0;
    const int D = 2 * M + 1;
    for (int j = 0; j < D * D; ++j) {
      const int dy = j / D - M, dx = j % D - M;
      const int r0 = wrap_index(r + dy, H), c0 = wrap_index(c + dx, W);
      const int c1 = c0 + 1 == W ? 0 : c0 + 1, r1 = r0 + 1 == H ? 0 : r0 + 1;
      for (int k = 0; k < K; ++k) {
        const T* zk = a.zprev + (size_t)k * n;
        const double z00 = (double)zk[(size_t)r0 * W + c0];
        const double gh = a.cw[j] * ((double)zk[(size_t)r0 * W + c1] - z00);
        const double gv = a.cw[j] * ((double)zk[(size_t)r1 * W + c0] - z00);
        A += gh * gh;
        B += gh * gv;
        C += gv * gv;
      }
    }
    const double hs = 0.5 * (A + C), hd = 0.5 * (A - C);
    const double R = sqrt(hd * hd + B * B);
    const double sp = sqrt(hs + R), sm = sqrt(fmax(hs - R, 0.0));
    const double nrm = a.pkind == kSchatten1   ? sp + sm
                       : a.pkind == kSchatten2 ? sqrt(fmax(A + C, 0.0))
                       : a.pkind == kSchattenP ? pow(pow(sp, a.pval) + pow(sm, a.pval), 1.0 / a.pval)
                                               : sp;
    val = -log(dot) + a.lambda * nrm;
  }
  const double t = block_sum(val, sh);
  if (threadIdx.x == 0) a.partial[blockIdx.x] = t;
}

// out[slot] = sum of partial[0..count) in index order.
__global__ void __launch_bounds__(256) reduce_kernel(const double* __restrict__ partial, int count, double* out,
                                                     int slot) {
  __shared__ double sh[4];
  double v = 0.0;
  // each thread sums a contiguous chunk, so the order is fixed for a given count
  const int per = (count + (int)blockDim.x - 1) / (int)blockDim.x;
  const int lo = threadIdx.x * per;
  for (int i = lo; i < lo + per && i < count; ++i) v += partial[i];
  const double t = block_sum(v, sh);
  if (threadIdx.x == 0) out[slot] = t;
}

template <typename T>
hipError_t launch_copy_t(const T* src, T* dst, size_t n, hipStream_t st) {
  size_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(copy_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}
hipError_t launch_copy(const float* s, float* d, size_t n, hipStream_t st) { return launch_copy_t(s, d, n, st); }
hipError_t launch_copy(const double* s, double* d, size_t n, hipStream_t st) { return launch_copy_t(s, d, n, st); }

template <typename T>
hipError_t launch_dual_res_t(const DiagArgs<T>& a, hipStream_t st) {
  hipLaunchKernelGGL(dual_res_kernel<T>, dim3(kDiagBlocks), dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(256), 0, st, a.partial, kDiagBlocks, a.out, 1);
  return hipGetLastError();
}
// Streaming copy: 16-byte nontemporal loads and stores, four per thread in
// flight, over a grid of a few workgroups per compute unit (the access
// pattern of the prox kernel's streaming build, without its arithmetic).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) stream_copy_kernel(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                          size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    u32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
  }
  for (; i < n; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 16;
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 256 * 8);
  hipLaunchKernelGGL(stream_copy_kernel, dim3(blocks), dim3(256), 0, st, reinterpret_cast<const u32x4*>(src),
                     reinterpret_cast<u32x4*>(dst), n);
  return hipGetLastError();
}

hipError_t launch_copy_bytes(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (bytes % 16 == 0)
    return launch_copy_t(reinterpret_cast<const uint4*>(src), reinterpret_cast<uint4*>(dst), bytes / 16, st);
  return launch_copy_t(reinterpret_cast<const unsigned char*>(src), reinterpret_cast<unsigned char*>(dst), bytes, st);
}

hipError_t launch_dual_res(const DiagArgs<float>& a, hipStream_t st) { return launch_dual_res_t(a, st); }
hipError_t launch_dual_res(const DiagArgs<double>& a, hipStream_t st) { return launch_dual_res_t(a, st); }

hipError_t launch_reduce(const double* partial, int count, double* out, int slot, hipStream_t st) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(256), 0, st, partial, count, out, slot);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_objective_t(const DiagArgs<T>& a, hipStream_t st) {
  const size_t n = (size_t)a.g.H * a.g.W;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(simplex_kernel<T>, dim3(blocks), dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(objective_kernel<T>, dim3(blocks), dim3(256), 0, st, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(256), 0, st, a.partial, (int)blocks, a.out, 2);
  return hipGetLastError();
}
hipError_t launch_objective(const DiagArgs<float>& a, hipStream_t st) { return launch_objective_t(a, st); }
hipError_t launch_objective(const DiagArgs<double>& a, hipStream_t st) { return launch_objective_t(a, st); }

}  // namespace segsalsa
