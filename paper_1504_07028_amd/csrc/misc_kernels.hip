// Set-up, initialisation, layout conversion and read-out kernels.
#include <cstring>
#include "segsalsa_internal.h"
#include "segsalsa_kernels.h"

namespace segsalsa {

// Twiddle tables exp(-2 pi i t / N) and the 1-D symbols 4 sin^2(pi t / N) of
// D^T D (periodic forward difference), in FP64 then rounded to T.
template <typename T>
__global__ void setup_kernel(const SetupArgs<T> a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < a.W) {
    double s, c;
    sincospi(2.0 * (double)t / (double)a.W, &s, &c);
    a.twW[t] = C2<T>{T(c), T(-s)};
    const double h = sinpi((double)t / (double)a.W);
    a.sx[t] = 4.0 * h * h;
  }
  if (t < a.H) {
    double s, c;
    sincospi(2.0 * (double)t / (double)a.H, &s, &c);
    a.twH[t] = C2<T>{T(c), T(-s)};
    const double h = sinpi((double)t / (double)a.H);
    a.sy[t] = 4.0 * h * h;
  }
  // Bluestein chirps, angle pi (t^2 mod 2N) / N, and power-of-two twiddles
  if (a.MW && t < a.W) {
    double s, c;
    sincospi((double)(((long long)t * t) % (2LL * a.W)) / (double)a.W, &s, &c);
    a.chW[t] = C2<T>{T(c), T(-s)};
  }
  if (a.MH && t < a.H) {
    double s, c;
    sincospi((double)(((long long)t * t) % (2LL * a.H)) / (double)a.H, &s, &c);
    a.chH[t] = C2<T>{T(c), T(-s)};
  }
  if (t < a.MW) {
    double s, c;
    sincospi(2.0 * (double)t / (double)a.MW, &s, &c);
    a.twMW[t] = C2<T>{T(c), T(-s)};
  }
  if (t < a.MH) {
    double s, c;
    sincospi(2.0 * (double)t / (double)a.MH, &s, &c);
    a.twMH[t] = C2<T>{T(c), T(-s)};
  }
  // fold lists (the host checked that none overflows)
  if (t < a.H) a.frow[t] = fold_list(a.g, t, true, a.frow + a.H + t, a.H);
  if (t < a.W) a.fcol[t] = fold_list(a.g, t, false, a.fcol + a.W + t, a.W);
}

template <typename T>
hipError_t launch_setup_t(const SetupArgs<T>& a, hipStream_t st) {
  int n = a.W > a.H ? a.W : a.H;
  n = n > a.MW ? n : a.MW;
  n = n > a.MH ? n : a.MH;
  hipLaunchKernelGGL(setup_kernel<T>, dim3((n + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}
hipError_t launch_setup(const SetupArgs<float>& a, hipStream_t st) { return launch_setup_t(a, st); }
hipError_t launch_setup(const SetupArgs<double>& a, hipStream_t st) { return launch_setup_t(a, st); }

// Initial state: p_hat = p / 1^T p (or softmax of logits), z = p_hat, d1 = d3 = d4 = 0.
template <typename T>
__global__ void init_kernel(const InitArgs<T> a) {
  const int H = a.g.H, W = a.g.W, K = a.K;
  const size_t n = (size_t)H * W;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int r = (int)(i / W), c = (int)(i - (size_t)r * W);
  int flags = 0;
  double mx = -1.0 / 0.0;
  double sum = 0.0;
  if (a.is_logits) {
    for (int k = 0; k < K; ++k) {
      const double x = (double)a.input[(size_t)k * n + i];
      if (!isfinite(x)) flags |= 1;
      mx = fmax(mx, x);
    }
    for (int k = 0; k < K; ++k) sum += exp((double)a.input[(size_t)k * n + i] - mx);
  } else {
    for (int k = 0; k < K; ++k) {
      const double x = (double)a.input[(size_t)k * n + i];
      if (!isfinite(x)) flags |= 1;
      if (x < 0.0) flags |= 2;
      sum += x;
    }
  }
  if (!(sum > 0.0)) flags |= 4;
  const double inv = 1.0 / sum;
  int tile, step, lane;
  tile_pos(a.g, r, c, tile, step, lane);
  const size_t sb = ((size_t)tile * a.g.steps + step) * K;
  for (int k = 0; k < K; ++k) {
    const double x = (double)a.input[(size_t)k * n + i];
    const T ph = T(a.is_logits ? exp(x - mx) * inv : x * inv);
    a.z[(size_t)k * n + i] = ph;
    a.phat[(sb + k) * 64 + lane] = ph;
    a.dm[((sb + k) * 3 + 0) * 64 + lane] = T(0);
    a.dm[((sb + k) * 3 + 1) * 64 + lane] = T(0);
    a.dm[((sb + k) * 3 + 2) * 64 + lane] = T(0);
  }
  if (flags) atomicOr(a.flags, flags);
}

template <typename T>
hipError_t launch_init_t(const InitArgs<T>& a, hipStream_t st) {
  const size_t n = (size_t)a.g.H * a.g.W;
  hipLaunchKernelGGL(init_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}
hipError_t launch_init(const InitArgs<float>& a, hipStream_t st) { return launch_init_t(a, st); }
hipError_t launch_init(const InitArgs<double>& a, hipStream_t st) { return launch_init_t(a, st); }

__global__ void fill_zero_kernel(uint4* p, size_t n16, unsigned char* tail, size_t ntail) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  const size_t n16 = bytes / 16;
  const size_t ntail = bytes - n16 * 16;
  size_t blocks = (n16 + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, reinterpret_cast<uint4*>(p), n16,
                     reinterpret_cast<unsigned char*>(p) + n16 * 16, ntail);
  return hipGetLastError();
}

struct StoreBlob {
  unsigned char b[2048];
};

__global__ void store_kernel(unsigned char* dst, StoreBlob blob, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = blob.b[i];
}

hipError_t launch_store(void* dst, const void* src, size_t n, hipStream_t st) {
  const unsigned char* s = reinterpret_cast<const unsigned char*>(src);
  unsigned char* d = reinterpret_cast<unsigned char*>(dst);
  for (size_t off = 0; off < n; off += sizeof(StoreBlob)) {
    StoreBlob blob;
    const size_t len = n - off < sizeof(StoreBlob) ? n - off : sizeof(StoreBlob);
    for (size_t i = 0; i < len; ++i) blob.b[i] = s[off + i];
    hipLaunchKernelGGL(store_kernel, dim3(1), dim3(256), 0, st, d + off, blob, (int)len);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

struct StorePair {
  unsigned char* dst[2];
  int n[2];
  unsigned char b[2][kStorePairMax];
};

__global__ void store_pair_kernel(StorePair sp) {
  for (int q = 0; q < 2; ++q)
    for (int i = threadIdx.x; i < sp.n[q]; i += blockDim.x) sp.dst[q][i] = sp.b[q][i];
}

hipError_t launch_store_pair(void* dst0, const void* src0, size_t n0, void* dst1, const void* src1, size_t n1,
                             hipStream_t st) {
  if (n0 > (size_t)kStorePairMax || n1 > (size_t)kStorePairMax) return hipErrorInvalidValue;
  StorePair sp;
  sp.dst[0] = reinterpret_cast<unsigned char*>(dst0);
  sp.dst[1] = reinterpret_cast<unsigned char*>(dst1);
  sp.n[0] = (int)n0;
  sp.n[1] = (int)n1;
  std::memcpy(sp.b[0], src0, n0);
  std::memcpy(sp.b[1], src1, n1);
  hipLaunchKernelGGL(store_pair_kernel, dim3(1), dim3(64), 0, st, sp);
  return hipGetLastError();
}

// Tile layout <-> canonical layouts, one thread per (pixel, class).
template <typename T>
__global__ void state_kernel(const StateArgs<T> a) {
  const int H = a.g.H, W = a.g.W, K = a.K, L = a.L;
  const size_t n = (size_t)H * W;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n * K) return;
  const int k = (int)(gid / n);
  const size_t i = gid - (size_t)k * n;
  const int r = (int)(i / W), c = (int)(i - (size_t)r * W);
  int tile, step, lane;
  tile_pos(a.g, r, c, tile, step, lane);
  const size_t kb = ((size_t)tile * a.g.steps + step) * K + k;
  const size_t ci = (size_t)k * n + i;
  if (a.to_canonical) {
    if (a.phat) a.phat[ci] = a.phat_t[kb * 64 + lane];
    if (a.d1) a.d1[ci] = a.dm_t[(kb * 3 + 0) * 64 + lane];
    if (a.d3) a.d3[ci] = a.dm_t[(kb * 3 + 1) * 64 + lane];
    if (a.d4) a.d4[ci] = a.dm_t[(kb * 3 + 2) * 64 + lane];
    if (a.d2) {
      for (int j = 0; j < L; ++j) {
        const C2<T> v = reinterpret_cast<const C2<T>*>(a.d2_t)[(kb * L + j) * 64 + lane];
        a.d2[((size_t)(j * 2 + 0) * K + k) * n + i] = v.x;
        a.d2[((size_t)(j * 2 + 1) * K + k) * n + i] = v.y;
      }
    }
  } else {
    a.phat_t[kb * 64 + lane] = a.phat[ci];
    a.dm_t[(kb * 3 + 0) * 64 + lane] = a.d1[ci];
    a.dm_t[(kb * 3 + 1) * 64 + lane] = a.d3[ci];
    a.dm_t[(kb * 3 + 2) * 64 + lane] = a.d4[ci];
    for (int j = 0; j < L; ++j) {
      C2<T> v;
      v.x = a.d2[((size_t)(j * 2 + 0) * K + k) * n + i];
      v.y = a.d2[((size_t)(j * 2 + 1) * K + k) * n + i];
      reinterpret_cast<C2<T>*>(a.d2_t)[(kb * L + j) * 64 + lane] = v;
    }
  }
}

template <typename T>
hipError_t launch_state_t(const StateArgs<T>& a, hipStream_t st) {
  const size_t tot = (size_t)a.g.H * a.g.W * a.K;
  hipLaunchKernelGGL(state_kernel<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}
hipError_t launch_state(const StateArgs<float>& a, hipStream_t st) { return launch_state_t(a, st); }
hipError_t launch_state(const StateArgs<double>& a, hipStream_t st) { return launch_state_t(a, st); }

// Segmentation read-out: argmax over classes, lowest class on ties.
template <typename T>
__global__ void labels_kernel(int K, size_t n, const T* __restrict__ z, int32_t* __restrict__ lab) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T best = z[i];
  int arg = 0;
  for (int k = 1; k < K; ++k) {
    const T v = z[(size_t)k * n + i];
    if (v > best) {
      best = v;
      arg = k;
    }
  }
  lab[i] = arg;
}

template <typename T>
hipError_t launch_labels_t(int K, int H, int W, const T* z, int32_t* lab, hipStream_t st) {
  const size_t n = (size_t)H * W;
  hipLaunchKernelGGL(labels_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, K, n, z, lab);
  return hipGetLastError();
}
hipError_t launch_labels(int K, int H, int W, const float* z, int32_t* lab, hipStream_t st) {
  return launch_labels_t(K, H, W, z, lab, st);
}
hipError_t launch_labels(int K, int H, int W, const double* z, int32_t* lab, hipStream_t st) {
  return launch_labels_t(K, H, W, z, lab, st);
}

}  // namespace segsalsa
