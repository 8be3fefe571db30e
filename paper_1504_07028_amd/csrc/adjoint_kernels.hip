// Reverse-mode sweep of the unrolled SALSA rounds of SegSALSA-STR (the
// adjoint of eqs. (12)-(14)): gradients of a loss of the final z with respect
// to the input, lambda and the patch multipliers c_j.
//
// One forward round maps (z, d1, d2, d3, d4) to (z', d') through
//   v_j = H_j z - d_j,  u_j = prox_j(v_j),  d'_j = u_j - v_j,
//   z' = A^{-1} G^T (u + d'),  A = 3 I + Wsum (D_h^T D_h + D_v^T D_v),
// where H_1 = H_3 = H_4 = I, H_2 = J and G^T (u + d') = sum_j H_j^T (2 u_j - v_j).
// Given the cotangents (zb', db') of the round's outputs, the reverse round is
//   rb  = A^{-1} zb'                               (the same FFT solve: A is symmetric)
//   ub_j = 2 H_j rb + db'_j
//   vb_j = -H_j rb - db'_j + (d prox_j / d v)^T ub_j
//   zb  = sum_j H_j^T vb_j,   db_j = -vb_j,
// plus the parameter terms
//   cb_j    += <vb_2,j, c_j^{-1} (J z)_j> + <c_j^{-1} (J rb)_j, 2 u_2,j - v_2,j>
//              - 2 c_j <D rb, D z'>        (J's entries, and Wsum in A)
//   lambdab += <ub_2, d u_2 / d tau> / mu  (tau = lambda / mu)
//   pb      += (d u_1 / d p)^T ub_1        (the data term's dependence on p)
// The proximity Jacobians are those of the closed forms of the forward pass:
//   g1: u = v + g p with g = 1/(mu t): du/dv = I + g_s p p^T, g_s = -g / disc
//   g2: U = Y N(S): Yb = Ub N + 2 Y Sb with Sb from the spectral derivative
//   g3: du/dv = [v > 0]            g4: du/dv = I - 1 1^T / K
// The kernel mirrors the forward one: a workgroup per tile, a wavefront per
// class, a lane per pixel, and the J^T scatter of the cotangent into the
// grown-tile accumulator that the FFT passes fold and solve.
#include "segsalsa_internal.h"
#include "segsalsa_kernels.h"
#include "prox_math.h"

namespace segsalsa {

template <typename T, int M, int KPW>
__global__ void __launch_bounds__((adj_max_threads<T, M, KPW>()), (adj_min_waves<T, M, KPW>())) adj_prox_kernel(const AdjArgs<T> a) {
  constexpr int D = 2 * M + 1;
  constexpr int L = D * D;
  constexpr int NS = 10;  // cross-class sums per pixel
  const TileGeom& g = a.g;
  const int tile = xcd_block();   // neighbouring tiles (shared halo rows) on one XCD
  const int tr = tile / g.ntc;
  const int tc = tile - tr * g.ntc;
  const int r0 = g.r0(tr), c0 = g.c0(tc);
  const int th = g.th(tr), tw = g.tw(tc);
  const int ER = th + 2 * M + 1, EC = tw + 2 * M + 1;
  const int plane = ER * EC;
  const int K = a.K, nw = a.nw;
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int H = g.H, W = g.W;

  extern __shared__ __align__(16) unsigned char smem[];
  T* zt = reinterpret_cast<T*>(smem);  // [K][ER][EC] z before the round
  T* rt = zt + K * plane;              // [K][ER][EC] rb = A^{-1} zb'
  T* acc = rt + K * plane;             // [K][ER][EC] partial sums of zb
  // offsets from smem (not integer casts of pointers) keep these accesses LDS instructions
  T* part = reinterpret_cast<T*>(smem + (((size_t)3 * K * plane * sizeof(T) + 15) & ~size_t(15)));
  // [NS][64] FP64 per-pixel class sums and [10][64] FP64 per-pixel coefficients
  double* tot = reinterpret_cast<double*>(part + 2 * NS * nw * 64);
  double* coef = tot + NS * 64;

  // z and rb over the grown tile, four elements per thread in flight at a
  // time (a plain strided loop waits for each load before issuing the next)
  const int ntot = K * plane;
  for (int i0 = threadIdx.x; i0 < ntot; i0 += 4 * blockDim.x) {
    T vz[4], vr[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = i0 + u * blockDim.x;
      vz[u] = vr[u] = T(0);
      if (idx < ntot) {
        const int k = idx / plane;
        const int rem = idx - k * plane;
        const int er = rem / EC, ec = rem - er * EC;
        const int gr = wrap_index(r0 - M + er, H), gc = wrap_index(c0 - M + ec, W);
        const size_t gi = ((size_t)k * H + gr) * W + gc;
        vz[u] = a.z[gi];
        vr[u] = a.r[gi];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = i0 + u * blockDim.x;
      if (idx < ntot) {
        zt[idx] = vz[u];
        rt[idx] = vr[u];
        acc[idx] = T(0);
      }
    }
  }
  __syncthreads();

  const int P = th * tw;
  const int nsteps = (P + 63) >> 6;
  // per-lane parameter sums over the tile's pixels and the wavefront's
  // classes: FP64 for FP64, FP32 for FP32 (a few dozen terms per lane,
  // reduced across lanes and tiles in FP64; half the registers)
  using Acc = typename std::conditional<sizeof(T) == 4, float, double>::type;
  Acc cb[L];
#pragma unroll
  for (int j = 0; j < L; ++j) cb[j] = Acc(0);
  Acc wb = Acc(0);
  double lb = 0.0;
  for (int s = 0; s < nsteps; ++s) {
    const int f = (s << 6) + lane;
    const bool valid = f < P;
    const int lr = valid ? f / tw : 0;
    const int lc = valid ? f - lr * tw : 0;
    const size_t stepbase = ((size_t)tile * g.steps + s) * K;

    T Y[KPW][L][2];
    T pk[KPW], v1[KPW], v3[KPW], rc[KPW], b1[KPW], b3[KPW];
    T ps = T(0), pq = T(0), pu = T(0), su4 = T(0), pa = T(0), pb = T(0), pc = T(0), q11 = T(0), q12 = T(0),
      q22 = T(0);
#pragma unroll
    for (int kk = 0; kk < KPW; ++kk) {
      const int k = wid + kk * nw;
      pk[kk] = v1[kk] = v3[kk] = rc[kk] = b1[kk] = b3[kk] = T(0);
      if (k < K && valid) {
        const size_t kb = stepbase + k;
        pk[kk] = a.phat[kb * 64 + lane];
        const T d1 = a.dm[(kb * 3 + 0) * 64 + lane];
        const T d3 = a.dm[(kb * 3 + 1) * 64 + lane];
        b1[kk] = a.bdm[(kb * 3 + 0) * 64 + lane];
        b3[kk] = a.bdm[(kb * 3 + 1) * 64 + lane];
        const T b4 = a.bdm[(kb * 3 + 2) * 64 + lane];
        const T* zk = zt + k * plane + (lr + M) * EC + (lc + M);
        const T* rk = rt + k * plane + (lr + M) * EC + (lc + M);
        const T zc = zk[0];
        rc[kk] = rk[0];
        v1[kk] = zc - d1;
        v3[kk] = zc - d3;
        ps += pk[kk] * v1[kk];
        pq += pk[kk] * pk[kk];
        pu += pk[kk] * (T(2) * rc[kk] + b1[kk]);
        su4 += T(2) * rc[kk] + b4;
        const C2<T>* d2p = reinterpret_cast<const C2<T>*>(a.d2) + kb * (size_t)(L * 64) + lane;
        const C2<T>* b2p = reinterpret_cast<const C2<T>*>(a.bd2) + kb * (size_t)(L * 64) + lane;
#pragma unroll
        for (int j = 0; j < L; ++j) {
          const int dy = j / D - M, dx = j % D - M;
          const T* zr = zk + dy * EC + dx;
          const T* rr = rk + dy * EC + dx;
          const C2<T> dd = d2p[j * 64];
          const C2<T> bb = b2p[j * 64];
          const T yh = a.c[j] * (zr[1] - zr[0]) - dd.x;
          const T yv = a.c[j] * (zr[EC] - zr[0]) - dd.y;
          const T uh = T(2) * (a.c[j] * (rr[1] - rr[0])) + bb.x;
          const T uv = T(2) * (a.c[j] * (rr[EC] - rr[0])) + bb.y;
          Y[kk][j][0] = yh;
          Y[kk][j][1] = yv;
          pa += yh * yh;
          pb += yh * yv;
          pc += yv * yv;
          q11 += yh * uh;
          q22 += yv * uv;
          q12 += yh * uv + yv * uh;
        }
      }
    }
    T* pbuf = part + (size_t)(s & 1) * NS * nw * 64;
    const T mine[NS] = {ps, pq, pu, su4, pa, pb, pc, q11, q12, q22};
#pragma unroll
    for (int q = 0; q < NS; ++q) pbuf[(q * nw + wid) * 64 + lane] = mine[q];
    __syncthreads();
    // class sums reduced once (wave q < NS takes sum q), the per-pixel FP64
    // closed forms evaluated once (waves 0 and 1) and shared through LDS
#pragma unroll 1
    for (int q = wid; q < NS; q += nw) {
      double t = 0.0;
#pragma unroll 1
      for (int w = 0; w < nw; ++w) t += (double)pbuf[(q * nw + w) * 64 + lane];
      tot[q * 64 + lane] = t;
    }
    __syncthreads();
    // the closed forms on three wavefronts: g1 and its derivatives, the
    // Schatten multiplier N, and its vector-Jacobian product (each recomputes
    // the eigenvalues; in parallel the FP64 phase is as long as its longest part)
    const int wn = nw > 1 ? 1 : 0;
    const int wv = nw > 2 ? 2 : wn;
    if (wid == 0 && valid) {
      const double S = tot[0 * 64 + lane], Q = tot[1 * 64 + lane], PU = tot[2 * 64 + lane];
      // g1: gain and its partial derivatives in s = p^T v and q = ||p||^2
      const double gain = data_prox_gain(S, Q, a.mu);
      const double disc = sqrt(S * S + 4.0 * Q / a.mu);
      const double gs = -gain / disc;
      const double gq = -gain * gain / disc;
      coef[0 * 64 + lane] = gain;
      coef[1 * 64 + lane] = gs * PU;
      coef[2 * 64 + lane] = 2.0 * gq * PU;
      coef[3 * 64 + lane] = tot[3 * 64 + lane] / (double)K;
    }
    if (wid == wn && valid) {  // g2: multiplier N
      double n11, n12, n22;
      schatten_multiplier<false>(tot[4 * 64 + lane], tot[5 * 64 + lane], tot[6 * 64 + lane], a.tau, a.pkind, 0.0,
                                 n11, n12, n22);
      coef[4 * 64 + lane] = n11;
      coef[5 * 64 + lane] = n12;
      coef[6 * 64 + lane] = n22;
    }
    if (wid == wv && valid) {  // g2: the cotangent of S and of tau
      double s11, s12, s22, dtau;
      schatten_multiplier_vjp(tot[4 * 64 + lane], tot[5 * 64 + lane], tot[6 * 64 + lane], a.tau, a.pkind,
                              tot[7 * 64 + lane], 0.5 * tot[8 * 64 + lane], tot[9 * 64 + lane], s11, s12, s22, dtau);
      lb += dtau;
      coef[7 * 64 + lane] = 2.0 * s11;
      coef[8 * 64 + lane] = 2.0 * s12;
      coef[9 * 64 + lane] = 2.0 * s22;
    }
    __syncthreads();
    if (valid) {
      const double gain = coef[0 * 64 + lane];
      const double pgs = coef[1 * 64 + lane];   // (p^T ub1) g_s
      const double pgq2 = coef[2 * 64 + lane];  // 2 (p^T ub1) g_q
      const T mean4 = T(coef[3 * 64 + lane]);
      const T m11 = T(coef[4 * 64 + lane]), m12 = T(coef[5 * 64 + lane]), m22 = T(coef[6 * 64 + lane]);
      const T t11 = T(coef[7 * 64 + lane]), t12 = T(coef[8 * 64 + lane]), t22 = T(coef[9 * 64 + lane]);
      const T kg = T(pgs);
      const int gr = r0 + lr, gc = c0 + lc;
      const size_t ic = (size_t)gr * W + gc;
      const size_t irr = (size_t)gr * W + (gc + 1 == W ? 0 : gc + 1);
      const size_t idn = (size_t)(gr + 1 == H ? 0 : gr + 1) * W + gc;

#pragma unroll
      for (int kk = 0; kk < KPW; ++kk) {
        const int k = wid + kk * nw;
        if (k < K) {
          const size_t kb = stepbase + k;
          const T r = rc[kk];
          const T vb1 = r + kg * pk[kk];
          const T vb3 = v3[kk] > T(0) ? r : -r - b3[kk];
          const T vb4 = r - mean4;
          const double u1b = 2.0 * (double)r + (double)b1[kk];
          a.pbar[kb * 64 + lane] += T(gain * u1b + pgs * (double)v1[kk] + pgq2 * (double)pk[kk]);
          a.bdm[(kb * 3 + 0) * 64 + lane] = -vb1;
          a.bdm[(kb * 3 + 1) * 64 + lane] = -vb3;
          a.bdm[(kb * 3 + 2) * 64 + lane] = -vb4;
          const T own = vb1 + vb3 + vb4;
          const T* zk = zt + k * plane + (lr + M) * EC + (lc + M);
          const T* rk = rt + k * plane + (lr + M) * EC + (lc + M);
          {  // <D rb, D z'> at this pixel and class (the Wsum term of A)
            const T* zn = a.zn + (size_t)k * H * W;
            const T znc = zn[ic];
            wb += (Acc)(rk[1] - rk[0]) * (Acc)(zn[irr] - znc) + (Acc)(rk[EC] - rk[0]) * (Acc)(zn[idn] - znc);
          }
          C2<T>* b2p = reinterpret_cast<C2<T>*>(a.bd2) + kb * (size_t)(L * 64) + lane;
          // Cotangent of Y per offset and its J^T scatter, destinations walked
          // in row-major order as in the forward kernel (same carries).
          T* ak = acc + k * plane + (lr + M) * EC + (lc + M);
          T vprev[D + 1];
#pragma unroll
          for (int q = 0; q <= D; ++q) vprev[q] = T(0);
#pragma unroll
          for (int da = -M; da <= M + 1; ++da) {
            T hprev = T(0);
#pragma unroll
            for (int db = -M; db <= M + 1; ++db) {
              const bool in0 = da <= M && db <= M;
              T ah = T(0), av = T(0);
              if (in0) {
                const int jj = (da + M) * D + (db + M);
                const T yh = Y[kk][jj][0], yv = Y[kk][jj][1];
                const T* zr = zk + da * EC + db;
                const T* rr = rk + da * EC + db;
                const T gzh = zr[1] - zr[0], gzv = zr[EC] - zr[0];
                const T grh = rr[1] - rr[0], grv = rr[EC] - rr[0];
                const T gh = a.c[jj] * grh, gv = a.c[jj] * grv;
                const C2<T> bb = b2p[jj * 64];
                const T uh = T(2) * gh + bb.x, uv = T(2) * gv + bb.y;
                const T ybh = uh * m11 + uv * m12 + (yh * t11 + yv * t12) - gh - bb.x;
                const T ybv = uh * m12 + uv * m22 + (yh * t12 + yv * t22) - gv - bb.y;
                C2<T> o;
                o.x = -ybh;
                o.y = -ybv;
                b2p[jj * 64] = o;
                const T a2h = T(2) * (yh * m11 + yv * m12) - yh;
                const T a2v = T(2) * (yh * m12 + yv * m22) - yv;
                cb[jj] += (Acc)ybh * (Acc)gzh + (Acc)ybv * (Acc)gzv + (Acc)grh * (Acc)a2h +
                          (Acc)grv * (Acc)a2v;
                ah = a.c[jj] * ybh;
                av = a.c[jj] * ybv;
              }
              const bool inh = da <= M && db - 1 >= -M;
              const bool inv = da - 1 >= -M && db <= M;
              const bool own_here = da == 0 && db == 0;
              const int q = db + M;
              if (in0 || inh || inv || own_here) {
                T gsum = own_here ? own : T(0);
                if (in0) gsum -= ah + av;
                if (inh) gsum += hprev;
                if (inv) gsum += vprev[q];
                if constexpr (sizeof(T) == 4 && M <= 3) {
                  volatile __attribute__((address_space(3))) T* at =
                      (volatile __attribute__((address_space(3))) T*)(ak + da * EC + db);
                  *at = *at + gsum;
                } else {
                  atomicAdd(ak + da * EC + db, gsum);
                }
              }
              hprev = ah;
              if (q <= D) vprev[q] = av;
            }
          }
        }
      }
    }  // valid
  }
  __syncthreads();
  // Per-tile parameter cotangents: wavefront sums, then waves in index order,
  // added to the tile's running totals (one workgroup per tile per launch, so
  // the order over rounds is fixed as well).
  double* red = reinterpret_cast<double*>(part);
  constexpr int NQ = L + 2;
  for (int q = 0; q < NQ; ++q) {
    double v = q < L ? (double)cb[q] : (q == L ? lb : (double)wb);
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) red[q * nw + wid] = v;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < NQ; q += blockDim.x) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[q * nw + w];
    a.gpart[(size_t)tile * NQ + q] += t;
  }
  T* blk = a.acc + (size_t)tile * K * g.ER * g.EC;
  for (int idx = threadIdx.x; idx < K * plane; idx += blockDim.x) {
    const int k = idx / plane;
    const int rem = idx - k * plane;
    const int er = rem / EC, ec = rem - er * EC;
    blk[((size_t)k * g.ER + er) * g.EC + ec] = acc[idx];
  }
}

// zb of the final z enters the reverse sweep as the grown-tile partial sums
// whose fold is zb itself: each pixel at its own tile's interior position.
template <typename T>
__global__ void __launch_bounds__(256) adj_load_kernel(const AdjIOArgs<T> a) {
  const int H = a.g.H, W = a.g.W, K = a.K, M = a.g.M;
  const size_t n = (size_t)H * W;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int r = (int)(i / W), c = (int)(i - (size_t)r * W);
  const int tr = a.g.trow(r), tc = a.g.tcol(c);
  const size_t tile = (size_t)tr * a.g.ntc + tc;
  const int er = r - a.g.r0(tr) + M, ec = c - a.g.c0(tc) + M;
  for (int k = 0; k < K; ++k)
    a.acc[((tile * K + k) * a.g.ER + er) * a.g.EC + ec] = a.grad_z[(size_t)k * n + i];
}

// Cotangent of the input: pb_total = fold(acc) (the cotangent of z^0 = p_hat)
// + the accumulated data-term part, pushed through the normalisation
// p_hat = x / 1^T x or p_hat = softmax(x):
//   x / 1^T x:  xb_k = (pb_k - <pb, p_hat>) / 1^T x
//   softmax:    xb_k = p_hat_k (pb_k - <pb, p_hat>)
template <typename T>
__global__ void __launch_bounds__(256) adj_input_kernel(const AdjIOArgs<T> a) {
  const int H = a.g.H, W = a.g.W, K = a.K;
  const size_t n = (size_t)H * W;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int r = (int)(i / W), c = (int)(i - (size_t)r * W);
  int tile, step, lane;
  tile_pos(a.g, r, c, tile, step, lane);
  const size_t sb = ((size_t)tile * a.g.steps + step) * K;
  const size_t plane = (size_t)a.g.ER * a.g.EC;
  const int* rl = a.frow + r;   // [kFoldStride][H]: count, then the entries
  const int* cl = a.fcol + c;
  auto folded = [&](int k) {
    T s = T(0);
    for (int u = 0; u < rl[0]; ++u) {
      const int ri = rl[(size_t)(1 + u) * H];
      for (int v = 0; v < cl[0]; ++v) {
        const int ci = cl[(size_t)(1 + v) * W];
        const size_t t = (size_t)(ri >> kFoldShift) * a.g.ntc + (ci >> kFoldShift);
        s += a.acc[(t * K + k) * plane + (size_t)(ri & kFoldMask) * a.g.EC + (ci & kFoldMask)];
      }
    }
    return (double)s + (double)a.pbar[(sb + k) * 64 + lane];
  };
  double dot = 0.0, sum = 0.0;
  for (int k = 0; k < K; ++k) {
    dot += folded(k) * (double)a.phat[(sb + k) * 64 + lane];
    if (!a.is_logits) sum += (double)a.input[(size_t)k * n + i];
  }
  for (int k = 0; k < K; ++k) {
    const double pbk = folded(k);
    const double ph = (double)a.phat[(sb + k) * 64 + lane];
    a.grad_input[(size_t)k * n + i] = T(a.is_logits ? ph * (pbk - dot) : (pbk - dot) / sum);
  }
}

// Final parameter gradients from the per-tile totals (fixed order over tiles):
//   grad_weights_j = cb_j - 2 c_j sum <D rb, D z'>,  grad_lambda = lb / mu.
__global__ void __launch_bounds__(128) adj_params_kernel(const double* __restrict__ gpart, int ntiles, int L,
                                                         AdjParamOut o) {
  const int NQ = L + 2;
  for (int q = threadIdx.x; q < NQ; q += blockDim.x) {
    double t = 0.0;
    for (int i = 0; i < ntiles; ++i) t += gpart[(size_t)i * NQ + q];
    o.tot[q] = t;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < L; q += blockDim.x)
    if (o.grad_weights) o.grad_weights[q] = o.tot[q] - 2.0 * o.c[q] * o.tot[L + 1];
  if (threadIdx.x == 0 && o.grad_lambda) *o.grad_lambda = o.tot[L] / o.mu;
}

template <typename T, int M, int KPW>
static hipError_t launch_adj_t(const AdjArgs<T>& a, int blocks, int threads, size_t lds, hipStream_t st) {
  auto fn = adj_prox_kernel<T, M, KPW>;
  static bool lds_set = false;
  if (!lds_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kLdsMax);
    if (e != hipSuccess) return e;
    lds_set = true;
  }
  hipLaunchKernelGGL(fn, dim3(blocks), dim3(threads), lds, st, a);
  return hipGetLastError();
}

template <typename T, int M>
static hipError_t launch_adj_m(const AdjArgs<T>& a, int blocks, int threads, int kpw, size_t lds, hipStream_t st) {
  switch (kpw) {
    case 1: return launch_adj_t<T, M, 1>(a, blocks, threads, lds, st);
    case 2: return launch_adj_t<T, M, 2>(a, blocks, threads, lds, st);
    case 4: return launch_adj_t<T, M, 4>(a, blocks, threads, lds, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t launch_adj_any(const AdjArgs<T>& a, int blocks, int threads, int M, int kpw, size_t lds,
                                 hipStream_t st) {
  switch (M) {
    case 0: return launch_adj_m<T, 0>(a, blocks, threads, kpw, lds, st);
    case 1: return launch_adj_m<T, 1>(a, blocks, threads, kpw, lds, st);
    case 2: return launch_adj_m<T, 2>(a, blocks, threads, kpw, lds, st);
    case 3: return launch_adj_m<T, 3>(a, blocks, threads, kpw, lds, st);
    case 4: return launch_adj_m<T, 4>(a, blocks, threads, kpw, lds, st);
    case 5: return launch_adj_m<T, 5>(a, blocks, threads, kpw, lds, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_adj_prox(const AdjArgs<float>& a, int blocks, int threads, int M, int kpw, size_t lds,
                           hipStream_t st) {
  return launch_adj_any<float>(a, blocks, threads, M, kpw, lds, st);
}
hipError_t launch_adj_prox(const AdjArgs<double>& a, int blocks, int threads, int M, int kpw, size_t lds,
                           hipStream_t st) {
  return launch_adj_any<double>(a, blocks, threads, M, kpw, lds, st);
}

template <typename T>
static hipError_t launch_adj_io_t(const AdjIOArgs<T>& a, bool load, hipStream_t st) {
  const size_t n = (size_t)a.g.H * a.g.W;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (load) hipLaunchKernelGGL(adj_load_kernel<T>, dim3(blocks), dim3(256), 0, st, a);
  else hipLaunchKernelGGL(adj_input_kernel<T>, dim3(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}
hipError_t launch_adj_load(const AdjIOArgs<float>& a, hipStream_t st) { return launch_adj_io_t(a, true, st); }
hipError_t launch_adj_load(const AdjIOArgs<double>& a, hipStream_t st) { return launch_adj_io_t(a, true, st); }
hipError_t launch_adj_input(const AdjIOArgs<float>& a, hipStream_t st) { return launch_adj_io_t(a, false, st); }
hipError_t launch_adj_input(const AdjIOArgs<double>& a, hipStream_t st) { return launch_adj_io_t(a, false, st); }

hipError_t launch_adj_params(const double* gpart, int ntiles, int L, const AdjParamOut& o, hipStream_t st) {
  hipLaunchKernelGGL(adj_params_kernel, dim3(1), dim3(128), 0, st, gpart, ntiles, L, o);
  return hipGetLastError();
}

}  // namespace segsalsa
