// Complex arithmetic and register butterflies shared by the FFT kernels
// (fft_kernels.hip: any length; fft_pow2_kernels.hip: power-of-two lengths).
#pragma once

#include "segsalsa_internal.h"

namespace segsalsa {

// Every LDS buffer and table of the FFT kernels is passed with its address space spelled
// out (lptr: LDS, gptr: global): generic pointers would become FLAT
// instructions, which are slower and make every LDS wait also wait for the
// outstanding global loads.
template <typename T>
using lptr = __attribute__((address_space(3))) T*;

// Complex element loads and stores through those pointers, member by member
// (the implicit copy operations of C2 only bind to generic addresses).
template <typename P>
__device__ __forceinline__ auto ldc(P p) {
  using T = decltype(+p->x);
  return C2<T>{p->x, p->y};
}
template <typename P, typename V>
__device__ __forceinline__ void stc(P p, const V& v) {
  p->x = v.x;
  p->y = v.y;
}

// Fold of a row workgroup: the right-hand side of rows row0 .. row0 + nb - 1
// (classes k0 and k0 + 1) from the grown-tile partial sums, handed to
// store(rr, c, value) for every element (rr: row within the workgroup).
// Thread i takes elements i, i + blockDim, ... (at most EPT of them; blockDim
// EPT >= nb W), all gathered into registers before the first store so that
// their loads are in flight together.  With a.vfold, groups of kFoldVec<T>
// adjacent columns (fold_gather_vec; W is then a multiple of the group),
// element by element (fold_gather) otherwise.
template <typename T, int EPT, typename Store>
__device__ __forceinline__ void fold_rows(const RowFwdArgs<T>& a, int row0, int nb, int k0, bool has1, Store store) {
  const gptr<const T> acc = glob(a.acc);
  const gptr<const int> frow = glob(a.frow), fcol = glob(a.fcol);
  const int H = a.g.H, W = a.g.W;
  const FastDiv fW(W);
  const int nel = nb * W;
  if (a.vfold) {
    constexpr int V = kFoldVec<T>;
    constexpr int NG = (EPT + V - 1) / V;
    T s0[NG * V], s1[NG * V];
#pragma unroll
    for (int it = 0; it < NG; ++it) {
      const int idx = (threadIdx.x + it * blockDim.x) * V;
      if (idx < nel) {
        const int rr = (int)fW.div(idx), c = idx - rr * W;
        fold_gather_vec(acc, frow + (row0 + rr), H, c, a.g, a.K, k0, has1, s0 + it * V, s1 + it * V);
      }
    }
#pragma unroll
    for (int it = 0; it < NG; ++it) {
      const int idx = (threadIdx.x + it * blockDim.x) * V;
      if (idx < nel) {
        const int rr = (int)fW.div(idx), c = idx - rr * W;
#pragma unroll
        for (int j = 0; j < V; ++j) store(rr, c + j, C2<T>{s0[it * V + j], s1[it * V + j]});
      }
    }
  } else {
    T s0[EPT], s1[EPT];
#pragma unroll
    for (int it = 0; it < EPT; ++it) {
      const int idx = threadIdx.x + it * blockDim.x;
      s0[it] = s1[it] = T(0);
      if (idx < nel) {
        const int rr = (int)fW.div(idx), c = idx - rr * W;
        fold_gather(acc, frow + (row0 + rr), fcol + c, H, W, a.g, a.K, k0, has1, s0[it], s1[it]);
      }
    }
#pragma unroll
    for (int it = 0; it < EPT; ++it) {
      const int idx = threadIdx.x + it * blockDim.x;
      if (idx < nel) {
        const int rr = (int)fW.div(idx), c = idx - rr * W;
        store(rr, c, C2<T>{s0[it], s1[it]});
      }
    }
  }
}

template <typename T>
__device__ inline C2<T> cadd(C2<T> a, C2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ inline C2<T> csub(C2<T> a, C2<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ inline C2<T> cscale(C2<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T>
__device__ inline C2<T> cmul(C2<T> a, C2<T> b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
// multiply by +i (sg = +1) or -i (sg = -1)
template <typename T>
__device__ inline C2<T> cmuli(C2<T> a, T sg) { return {-sg * a.y, sg * a.x}; }
// a * w (forward) or a * conj(w) (inverse)
template <typename T>
__device__ inline C2<T> twmul(C2<T> a, C2<T> w, bool inv) {
  const T wy = inv ? -w.y : w.y;
  return {a.x * w.x - a.y * wy, a.x * wy + a.y * w.x};
}

// DFT of R values, y_q = sum_r v_r exp(sg 2 pi i r q / R), sg = -1 forward, +1 inverse.
template <typename T, int R>
struct Bfly;

template <typename T>
struct Bfly<T, 2> {
  __device__ static void run(C2<T>* v, T) {
    const C2<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <typename T>
struct Bfly<T, 3> {
  __device__ static void run(C2<T>* v, T sg) {
    const T h = T(0.86602540378443864676);  // sin(2 pi / 3)
    const C2<T> t = cadd(v[1], v[2]);
    const C2<T> d = csub(v[1], v[2]);
    const C2<T> m = {v[0].x - T(0.5) * t.x, v[0].y - T(0.5) * t.y};
    const C2<T> e = cmuli(cscale(d, h), sg);
    v[0] = cadd(v[0], t);
    v[1] = cadd(m, e);
    v[2] = csub(m, e);
  }
};

template <typename T>
struct Bfly<T, 4> {
  __device__ static void run(C2<T>* v, T sg) {
    const C2<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const C2<T> t2 = cadd(v[1], v[3]), t3 = cmuli(csub(v[1], v[3]), sg);
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

template <typename T>
struct Bfly<T, 5> {
  __device__ static void run(C2<T>* v, T sg) {
    const T c1 = T(0.30901699437494742410);   // cos(2 pi / 5)
    const T c2 = T(-0.80901699437494742410);  // cos(4 pi / 5)
    const T s1 = T(0.95105651629515357212);   // sin(2 pi / 5)
    const T s2 = T(0.58778525229247312917);   // sin(4 pi / 5)
    const C2<T> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    const C2<T> t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    const C2<T> b1 = {v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y};
    const C2<T> b2 = {v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y};
    const C2<T> e1 = cmuli(C2<T>{s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y}, sg);
    const C2<T> e2 = cmuli(C2<T>{s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y}, sg);
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = cadd(b1, e1);
    v[4] = csub(b1, e1);
    v[2] = cadd(b2, e2);
    v[3] = csub(b2, e2);
  }
};

template <typename T>
struct Bfly<T, 8> {
  __device__ static void run(C2<T>* v, T sg) {
    const T r = T(0.70710678118654752440);  // 1/sqrt(2)
    C2<T> e[4] = {v[0], v[2], v[4], v[6]};
    C2<T> o[4] = {v[1], v[3], v[5], v[7]};
    Bfly<T, 4>::run(e, sg);
    Bfly<T, 4>::run(o, sg);
    // o_q *= exp(sg 2 pi i q / 8)
    const C2<T> o1 = {r * (o[1].x - sg * o[1].y), r * (o[1].y + sg * o[1].x)};
    const C2<T> o2 = cmuli(o[2], sg);
    const C2<T> o3 = {r * (-o[3].x - sg * o[3].y), r * (-o[3].y + sg * o[3].x)};
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

}  // namespace segsalsa
