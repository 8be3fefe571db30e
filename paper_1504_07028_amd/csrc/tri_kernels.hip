// Column half of the z-update solve (eq. (12)) without a column DFT.
//
// After the row DFT, the operator A = 3 I + Wsum (D_h^T D_h + D_v^T D_v)
// acts on each column of spatial frequency kx as the periodic tridiagonal
// Toeplitz matrix T = a I - b (S + S^-1), a = 3 + Wsum (2 + 4 sin^2(pi kx / W)),
// b = Wsum, S the cyclic shift along the column.  With rho + 1/rho = a / b,
// 0 <= rho < 1 (a - 2b >= 3 > 0), it factors as
//   T = (b / rho) (I - rho S) (I - rho S^-1),
// so T^-1 r = (rho / b) v with u = r + rho S u (u_y = r_y + rho u_(y-1)) and
// v = u + rho S^-1 v (v_y = u_y + rho v_(y+1)), both periodic: two
// first-order recursions.  The result equals the DFT route's
// IDFT_y(DFT_y(r) / symbol) up to rounding, for every column length (no
// factorisation, no Bluestein) and every Wsum.
//
// Each column's H values are cut into chunks of LPT consecutive rows, one
// chunk per thread, in registers.  A recursion over a chunk started from 0
// gives the chunk's affine map (value after the chunk) = rho^len (value
// before) + offset; an inclusive scan of the maps over the chunks (in LDS,
// log2 steps) gives every chunk's incoming value in terms of the column's
// periodic closure, which the composition of all maps fixes exactly:
// x = A_all x + B_all, x = B_all / (1 - rho^H).  Each chunk then adds
// rho^k times its incoming value.  The backward recursion does the same from
// the other end.  The pass reads and writes the spectrum once.
//
// Lanes take consecutive columns first (cols_per_block of them), so a load
// or store of one row slot touches that many adjacent columns.  The
// workgroup holds at least cols_per_block * ceil(H / LPT) threads; a batch
// launches every column length with one workgroup size.
#include "segsalsa_internal.h"
#include "segsalsa_kernels.h"
#include "fft_math.h"

namespace segsalsa {

// f(x) = A x + B composed with g(x) = A2 x + B2: f(g(x))
template <typename T>
__device__ __forceinline__ void compose(T& A, C2<T>& B, T A2, C2<T> B2) {
  B = C2<T>{A * B2.x + B.x, A * B2.y + B.y};
  A = A * A2;
}

template <typename T, int LPT>
__global__ void __launch_bounds__(kFftMaxThreads) cols_tri_kernel(const ColArgs<T>* __restrict__ descs, int ndesc) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int blk = xcd_block();
  const ColArgs<T>& a = descs[find_desc(descs, ndesc, blk)];
  const int bid = blk - a.block0;
  const int H = a.H, W = a.W;
  const int cpb = a.cols_per_block;
  const int ncb = (W + cpb - 1) / cpb;
  const int m = bid / ncb;
  const FastDiv fc(cpb);
  const int t = (int)fc.div(threadIdx.x), j = threadIdx.x - t * cpb;
  const int tpc = (H + LPT - 1) / LPT;   // chunks per column; threads beyond cpb * tpc only join the barriers
  const int x = (bid - m * ncb) * cpb + j;
  const bool active = x < W && t < tpc;
  const int y0 = t * LPT;
  const int len = t < tpc ? min(LPT, H - y0) : 0;
  // coefficients of the column (FP64, then the working precision)
  T rho, gain;
  {
    const double wsum = a.wsum;
    const double aa = 3.0 + wsum * (2.0 + (x < W ? glob(a.sx)[x] : 0.0));
    const double den = aa + sqrt(fmax(aa * aa - 4.0 * wsum * wsum, 0.0));
    rho = T(2.0 * wsum / den);                  // the root of rho^2 - (a / b) rho + 1 = 0 below 1
    gain = T(2.0 / den / (double)W);            // rho / b, and the 1 / W of the row DFT
  }
  const gptr<C2<T>> sp = glob(a.spec) + (size_t)m * H * W + x;
  C2<T> v[LPT];
#pragma unroll
  for (int i = 0; i < LPT; ++i) v[i] = active && i < len ? ldc(sp + (size_t)(y0 + i) * W) : C2<T>{T(0), T(0)};
  T Achunk = T(1);   // rho^len
#pragma unroll
  for (int i = 0; i < LPT; ++i)
    if (i < len) Achunk *= rho;

  // LDS: two buffers of (A, B) per thread for the scans
  T* sA = reinterpret_cast<T*>(smem);
  C2<T>* sB = reinterpret_cast<C2<T>*>(smem + ((2 * blockDim.x * sizeof(T) + 15) & ~size_t(15)));
  const int n = blockDim.x;

  // inclusive scan of the chunk maps along the column, forward (dir = +1:
  // chunk t combines with t - d) or backward (dir = -1: with t + d); returns
  // the composition of all maps in (Atot, Btot) and the exclusive one in (Ax, Bx)
  auto scan = [&](T A, C2<T> B, int dir, T& Ax, C2<T>& Bx, T& Atot, C2<T>& Btot) {
    int cur = 0;
    sA[threadIdx.x] = A;
    sB[threadIdx.x] = B;
    __syncthreads();
    for (int d = 1; d < tpc; d <<= 1) {
      const int o = t - dir * d;
      if (o >= 0 && o < tpc) compose(A, B, sA[cur * n + o * cpb + j], sB[cur * n + o * cpb + j]);
      cur ^= 1;
      sA[cur * n + threadIdx.x] = A;
      sB[cur * n + threadIdx.x] = B;
      __syncthreads();
    }
    const int last = dir > 0 ? tpc - 1 : 0;
    Atot = sA[cur * n + last * cpb + j];
    Btot = sB[cur * n + last * cpb + j];
    const int prev = t - dir;
    if (prev >= 0 && prev < tpc) {
      Ax = sA[cur * n + prev * cpb + j];
      Bx = sB[cur * n + prev * cpb + j];
    } else {
      Ax = T(1);
      Bx = C2<T>{T(0), T(0)};
    }
    __syncthreads();   // every read done before the buffers are written again
  };

  // forward recursion u_y = r_y + rho u_(y-1)
  C2<T> u = {T(0), T(0)};
#pragma unroll
  for (int i = 0; i < LPT; ++i)
    if (i < len) {
      u = C2<T>{v[i].x + rho * u.x, v[i].y + rho * u.y};
      v[i] = u;
    }
  T Ax, Atot;
  C2<T> Bx, Btot;
  scan(Achunk, u, +1, Ax, Bx, Atot, Btot);
  {
    // u before row 0 is u_(H-1): the fixed point of the whole column's map
    const T s = T(1) / (T(1) - Atot);
    const C2<T> u0 = {Btot.x * s, Btot.y * s};
    const C2<T> uin = {Ax * u0.x + Bx.x, Ax * u0.y + Bx.y};   // u just before this chunk
    T p = rho;   // rho^(i + 1)
#pragma unroll
    for (int i = 0; i < LPT; ++i) {
      v[i].x += p * uin.x;
      v[i].y += p * uin.y;
      p *= rho;
    }
  }
  // backward recursion v_y = u_y + rho v_(y+1)
  C2<T> w = {T(0), T(0)};
#pragma unroll
  for (int i = LPT - 1; i >= 0; --i)
    if (i < len) {
      w = C2<T>{v[i].x + rho * w.x, v[i].y + rho * w.y};
      v[i] = w;
    }
  scan(Achunk, w, -1, Ax, Bx, Atot, Btot);
  {
    const T s = T(1) / (T(1) - Atot);
    const C2<T> v0 = {Btot.x * s, Btot.y * s};                   // v after row H - 1 is v_0
    const C2<T> vin = {Ax * v0.x + Bx.x, Ax * v0.y + Bx.y};      // v just after this chunk
    T p = rho;   // rho^(len - i)
#pragma unroll
    for (int i = LPT - 1; i >= 0; --i)
      if (i < len) {
        v[i].x = gain * (v[i].x + p * vin.x);
        v[i].y = gain * (v[i].y + p * vin.y);
        p *= rho;
      }
  }
  if (active) {
#pragma unroll
    for (int i = 0; i < LPT; ++i)
      if (i < len) stc(sp + (size_t)(y0 + i) * W, v[i]);
  }
}

template <typename T, int LPT>
static hipError_t launch_tri_t(const ColArgs<T>* d, int n, int blocks, int threads, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL((cols_tri_kernel<T, LPT>), dim3(blocks), dim3(threads), lds, st, d, n);
  return hipGetLastError();
}

hipError_t launch_cols_tri(const ColArgs<float>* d, int n, int blocks, int lpt, int threads, size_t lds,
                           hipStream_t st) {
  return lpt == 32 ? launch_tri_t<float, 32>(d, n, blocks, threads, lds, st)
                   : lpt == 16 ? launch_tri_t<float, 16>(d, n, blocks, threads, lds, st) : hipErrorInvalidValue;
}
hipError_t launch_cols_tri(const ColArgs<double>* d, int n, int blocks, int lpt, int threads, size_t lds,
                           hipStream_t st) {
  return lpt == 32 ? launch_tri_t<double, 32>(d, n, blocks, threads, lds, st)
                   : lpt == 16 ? launch_tri_t<double, 16>(d, n, blocks, threads, lds, st) : hipErrorInvalidValue;
}

}  // namespace segsalsa
