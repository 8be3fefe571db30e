// Power-of-two FFT engine with the transform structure fixed at compile
// time, for N = 64 ... 4096 points (the z-update's DFTs, eq. (12)).
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
#pragma once
#include "segsalsa_internal.h"
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

}  // namespace segsalsa
