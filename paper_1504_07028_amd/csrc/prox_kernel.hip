// Fused per-pixel proximity kernel of one SALSA round (SegSALSA-STR, Sec. 4).
//
// One workgroup owns one tile of the image.  Wavefront w handles classes
// k = w, w + nw, ... for 64 pixels at a time (one pixel per lane).  Per pixel
// and round it computes, from z and the scaled multipliers d:
//   g1 (data term, eq. (10)):   u1 = prox_{g1/mu}(z - d1): closed-form root
//                               of mu t^2 - mu (p^T v) t - ||p||^2 = 0
//   g2 (Schatten prior):        u2 = prox_{(lambda/mu)||.||_{S_p}}(J z - d2),
//                               reduced to the 2x2 structure tensor (eq. (5))
//   g3 (positivity):            u3 = max(z - d3, 0)
//   g4 (sum to one):            u4 = (z - d4) - (1^T (z - d4) - 1) / K, or, with
//                               g4s, the projection of z - d4 onto the probability
//                               simplex: u4 = max(v4 - theta, 0) with 1^T u4 = 1
// the multiplier update d_j <- u_j - (H_j z - d_j) (eq. (14)), and scatters
// u_j + d_j through H_j^T into a per-tile accumulator: the right-hand side
// G^T (u + d) of the normal equations of the z-update (eq. (12)).
//
// The J^T scatter of a pixel reaches pixels up to (M, M+1) away, so every
// tile accumulates over its tile grown by that margin in LDS; the row FFT
// pass sums the overlapping grown tiles.  A class's accumulator is written by
// one wavefront only and, within one instruction, lanes hit distinct
// addresses, so plain LDS read-modify-writes (in program order) are free of
// races and their summation order is fixed.
#include "segsalsa_internal.h"
#include "segsalsa_kernels.h"
#include "prox_math.h"

namespace segsalsa {

// VAR compiles in the method's variants (general Schatten p, simplex g4) and
// the primal-residual accumulation of checked rounds; the plain instantiation
// (p in {1, 2, inf}, affine g4, no residuals) stays lean.
//
// PF (prefetch): the loads of step s + 1 (p_hat, d1, d3, d4 and the raw d2
// pairs of the wavefront's classes) are issued into a second register set at
// the start of step s's multiplier/scatter phase, so that they stream while
// that phase computes and stores.  All wavefronts of a workgroup run each
// step's phases in lockstep (three barriers per step), and without it the
// loads of a step only start once the previous step's work is done, so the
// memory and the arithmetic of a step never overlap.  It doubles the per-lane
// state, hence fewer (and fuller) wavefronts.
//
// SY (streamed Y, patches of 9x9 and larger): the 2L values of Y = J z - d2
// of a pixel and class are not kept in registers between the structure-tensor
// sums and the update; the update phase rebuilds each offset's pair from z in
// LDS and the old d2 (read again, just before its new value overwrites it).
// The registers then do not grow with L, so these patches keep the wavefront
// count and the ordered FP32 scatter of the smaller ones, at the price of a
// second read of d2 (mostly served by the caches).
//
// NT (streaming, plain instantiation only): p_hat, d1, d3, d4 and d2 are
// loaded and stored nontemporally, and so are the grown-tile partial sums
// written at the end (measured: the fold that reads them next runs as fast or
// faster).  A round touches the state once, so when the state of all images
// of a launch far exceeds the L2s and the 256 MB MALL, caching it only evicts
// what the next kernels read again (z, the spectrum); when it fits, the
// cached accesses keep it resident from round to round.  The host chooses per
// round from the state's size.
template <typename T, int M, int KPW, bool VAR, bool PF, bool NT>
__global__ void __launch_bounds__((prox_max_threads<T, M, KPW, PF>()))
prox_rhs_kernel(const ProxArgs<T>* __restrict__ descs, int ndesc) {
  constexpr int D = 2 * M + 1;
  constexpr int L = D * D;
  constexpr bool SY = prox_streams_y<M>();
  constexpr int LY = SY ? 1 : L;
  const int blk = xcd_block();   // neighbouring tiles (shared halo rows) on one XCD
  const ProxArgs<T>& a = descs[find_desc(descs, ndesc, blk)];
  const TileGeom& g = a.g;
  const int tile = blk - a.block0;
  const int tr = tile / g.ntc;
  const int tc = tile - tr * g.ntc;
  const int r0 = g.r0(tr), c0 = g.c0(tc);
  const int th = g.th(tr), tw = g.tw(tc);
  const int ER = th + 2 * M + 1, EC = tw + 2 * M + 1;
  const int plane = ER * EC;
  const int K = a.K, nw = a.nw;
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int H = g.H, W = g.W;
  const bool g4s = VAR && a.g4s;
  const gptr<const T> gz = glob(a.z);
  const gptr<const T> gphat = glob(a.phat);
  const gptr<const T> gdm_in = glob(a.dm_in);
  const gptr<const T> gd2_in = glob(a.d2_in);   // (h, v) pairs
  const gptr<T> gdm = glob(a.dm);
  const gptr<T> gd2 = glob(a.d2);
  // NT: the per-pixel state streams past the caches (nontemporal loads and
  // stores), for rounds whose state is far larger than the caches
  auto sld = [](gptr<const T> p) -> T {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
  };
  auto sst = [](gptr<T> p, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
  };

  extern __shared__ __align__(16) unsigned char smem[];
  T* zt = reinterpret_cast<T*>(smem);  // [K][ER][EC] z over the grown tile (periodic)
  T* acc = zt + K * plane;             // [K][ER][EC] G^T(u + d) partial sums
  // [2][6][nw][64] per-class partial sums, 16-byte aligned (also read as doubles);
  // with g4s, after the FP64 sums and coefficients, [2][K][64] v4 of every
  // class (double-buffered by step like the sums)
  // (offsets from smem, not integer casts of pointers: the compiler then keeps
  // these accesses as LDS instructions instead of generic FLAT ones, which
  // would also wait for outstanding global memory operations)
  T* part = reinterpret_cast<T*>(smem + (((size_t)2 * K * plane * sizeof(T) + 15) & ~size_t(15)));
  // [6][64] FP64 per-pixel class sums and [5][64] FP64 per-pixel coefficients
  double* tot = reinterpret_cast<double*>(part + 2 * 6 * nw * 64);
  double* coef = tot + 6 * 64;
  T* v4buf = reinterpret_cast<T*>(coef + 5 * 64);

  // z over the grown tile, four loads per thread in flight at a time (a
  // plain strided loop waits for each load before issuing the next)
  const int ntot = K * plane;
  for (int i0 = threadIdx.x; i0 < ntot; i0 += 4 * blockDim.x) {
    T v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = i0 + u * blockDim.x;
      v[u] = T(0);
      if (idx < ntot) {
        const int k = idx / plane;
        const int rem = idx - k * plane;
        const int er = rem / EC, ec = rem - er * EC;
        const int gr = wrap_index(r0 - M + er, H), gc = wrap_index(c0 - M + ec, W);
        v[u] = gz[((size_t)k * H + gr) * W + gc];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = i0 + u * blockDim.x;
      if (idx < ntot) {
        zt[idx] = v[u];
        acc[idx] = T(0);
      }
    }
  }
  __syncthreads();

  const int P = th * tw;
  const int nsteps = (P + 63) >> 6;
  const bool want_res = VAR && a.res_tile != nullptr;  // checked rounds use the VAR instantiation
  double rp_acc = 0.0;
  // prefetched inputs of the next step (PF)
  constexpr int KP = PF ? KPW : 1, LP = PF ? L : 1;
  T Pp[KP], P1[KP], P3[KP], P4[KP], Pd[KP][LP][2];
  // class kk's inputs of step sn (one class at a time, so that in the update
  // phase the next step's block of a class only becomes live as the current
  // step's block of the class before it dies)
  auto prefetch = [&](int sn, int kk) {
    const bool vn = (sn << 6) + lane < P;
    const int k = wid + kk * nw;
    if (k < K && vn) {
      const size_t kb = ((size_t)tile * g.steps + sn) * K + k;
      Pp[kk] = gphat[kb * 64 + lane];
      P1[kk] = gdm_in[(kb * 3 + 0) * 64 + lane];
      P3[kk] = gdm_in[(kb * 3 + 1) * 64 + lane];
      P4[kk] = gdm_in[(kb * 3 + 2) * 64 + lane];
      const gptr<const T> d2p = gd2_in + 2 * (kb * (size_t)(L * 64) + lane);
#pragma unroll
      for (int j = 0; j < LP; ++j) {
        Pd[kk][j][0] = d2p[j * 128];
        Pd[kk][j][1] = d2p[j * 128 + 1];
      }
    }
  };
  if constexpr (PF) {
#pragma unroll
    for (int kk = 0; kk < KP; ++kk) prefetch(0, kk);
  }
  for (int s = 0; s < nsteps; ++s) {
    const int f = (s << 6) + lane;
    const bool valid = f < P;
    const int lr = valid ? f / tw : 0;
    const int lc = valid ? f - lr * tw : 0;
    const size_t stepbase = ((size_t)tile * g.steps + s) * K;

    T Y[KPW][LY][2];
    T pk[KPW], v1[KPW], v3[KPW], v4[KPW];
    T ps = T(0), pq = T(0), psv = T(0), pa = T(0), pb = T(0), pc = T(0);
#pragma unroll
    for (int kk = 0; kk < KPW; ++kk) {
      const int k = wid + kk * nw;
      pk[kk] = v1[kk] = v3[kk] = v4[kk] = T(0);
      if (k < K && valid) {
        const size_t kb = stepbase + k;
        T d1, d3, d4;
        if constexpr (PF) {
          pk[kk] = Pp[kk];
          d1 = P1[kk];
          d3 = P3[kk];
          d4 = P4[kk];
        } else {
          pk[kk] = sld(gphat + kb * 64 + lane);
          d1 = sld(gdm_in + (kb * 3 + 0) * 64 + lane);
          d3 = sld(gdm_in + (kb * 3 + 1) * 64 + lane);
          d4 = sld(gdm_in + (kb * 3 + 2) * 64 + lane);
        }
        const T* zk = zt + k * plane + (lr + M) * EC + (lc + M);
        const T zc = zk[0];
        v1[kk] = zc - d1;
        v3[kk] = zc - d3;
        v4[kk] = zc - d4;
        ps += pk[kk] * v1[kk];
        pq += pk[kk] * pk[kk];
        psv += v4[kk];
        if (g4s) v4buf[((s & 1) * K + k) * 64 + lane] = v4[kk];
        const gptr<const T> d2p = gd2_in + 2 * (kb * (size_t)(L * 64) + lane);
#pragma unroll
        for (int j = 0; j < L; ++j) {
          const int dy = j / D - M, dx = j % D - M;
          const T* zr = zk + dy * EC + dx;
          const T z00 = zr[0], z01 = zr[1], z10 = zr[EC];
          C2<T> dd;
          if constexpr (PF) {
            dd.x = Pd[kk][j < LP ? j : 0][0];
            dd.y = Pd[kk][j < LP ? j : 0][1];
          } else {
            // (the streamed-Y patches read d2 again in the update: cached)
            dd.x = SY ? d2p[j * 128] : sld(d2p + j * 128);
            dd.y = SY ? d2p[j * 128 + 1] : sld(d2p + j * 128 + 1);
          }
          const T yh = a.c[j] * (z01 - z00) - dd.x;
          const T yv = a.c[j] * (z10 - z00) - dd.y;
          if constexpr (!SY) {
            Y[kk][j][0] = yh;
            Y[kk][j][1] = yv;
          }
          pa += yh * yh;
          pb += yh * yv;
          pc += yv * yv;
        }
      }
    }
    // Per-pixel sums over the classes and the per-pixel coefficients, each
    // computed once per step: waves q < 6 reduce the q-th sum over the
    // wavefronts in FP64, then waves 0 and 1 evaluate the two FP64 closed
    // forms and share them through LDS (the other wavefronts would only
    // repeat them: the per-step VALU work is what bounds this kernel).
    T* pbuf = part + (size_t)(s & 1) * 6 * nw * 64;
    pbuf[(0 * nw + wid) * 64 + lane] = ps;
    pbuf[(1 * nw + wid) * 64 + lane] = pq;
    pbuf[(2 * nw + wid) * 64 + lane] = psv;
    pbuf[(3 * nw + wid) * 64 + lane] = pa;
    pbuf[(4 * nw + wid) * 64 + lane] = pb;
    pbuf[(5 * nw + wid) * 64 + lane] = pc;
    __syncthreads();
#pragma unroll 1
    for (int q = wid; q < 6; q += nw) {
      double t = 0.0;  // fixed order w = 0, 1, ...; unrolled so the LDS reads overlap
#pragma unroll 4
      for (int w = 0; w < nw; ++w) t += (double)pbuf[(q * nw + w) * 64 + lane];
      tot[q * 64 + lane] = t;
    }
    __syncthreads();
    // the two FP64 closed forms on two different wavefronts (each keeps its
    // own class block live, so splitting them keeps the register peak down)
    const int wn = nw > 1 ? 1 : 0;
    if (wid == 0 && valid) {
      const double S = tot[0 * 64 + lane], Q = tot[1 * 64 + lane], SV = tot[2 * 64 + lane];
      double g4c = -(SV - 1.0) / (double)K;  // affine g4: the shared d4 of the pixel
      if (g4s) {
        // simplex g4: threshold theta with sum_k max(v4_k - theta, 0) = 1, by
        // Michelot's active-set iteration (theta rises, the active set
        // shrinks, at most K passes over the pixel's K values)
        const T* vb = v4buf + (size_t)(s & 1) * K * 64 + lane;
        double theta = (SV - 1.0) / (double)K;
        int cnt = K;
        for (int it = 0; it < K; ++it) {
          double sum = 0.0;
          int c2 = 0;
          for (int k = 0; k < K; ++k) {
            const double v = (double)vb[k * 64];
            if (v > theta) {
              sum += v;
              ++c2;
            }
          }
          if (c2 == cnt || c2 == 0) break;
          cnt = c2;
          theta = (sum - 1.0) / (double)c2;
        }
        g4c = theta;
      }
      coef[0 * 64 + lane] = data_prox_gain(S, Q, a.mu);
      coef[1 * 64 + lane] = g4c;
    }
    if (wid == wn && valid) {
      const double A = tot[3 * 64 + lane], B = tot[4 * 64 + lane], C = tot[5 * 64 + lane];
      double n11, n12, n22;
      schatten_multiplier<VAR>(A, B, C, a.tau, a.pkind, a.pval, n11, n12, n22);
      coef[2 * 64 + lane] = n11 - 1.0;
      coef[3 * 64 + lane] = n12;
      coef[4 * 64 + lane] = n22 - 1.0;
    }
    __syncthreads();
    // (with PF, the next step's loads are issued class by class below: a step
    // other than the last has all its lanes valid, so they are issued by every lane)
    if (valid) {
    const double gain = coef[0 * 64 + lane];
    const double g4c = coef[1 * 64 + lane];
    const T d4a = T(g4c);
    const double theta = g4c;
    const T m11 = T(coef[2 * 64 + lane]), m12 = T(coef[3 * 64 + lane]), m22 = T(coef[4 * 64 + lane]);

#pragma unroll
    for (int kk = 0; kk < KPW; ++kk) {
      const int k = wid + kk * nw;
      if constexpr (PF) {
        if (s + 1 < nsteps) prefetch(s + 1, kk);   // streams while this class's updates compute and store
      }
      if (k < K) {
        const size_t kb = stepbase + k;
        const T d1n = T((double)pk[kk] * gain);
        const T d3n = v3[kk] < T(0) ? -v3[kk] : T(0);
        const T d4n = g4s ? T(fmax((double)v4[kk] - theta, 0.0) - (double)v4[kk]) : d4a;
        const T own = (v1[kk] + T(2) * d1n) + (v3[kk] < T(0) ? -v3[kk] : v3[kk]) + (v4[kk] + T(2) * d4n);
        sst(gdm + (kb * 3 + 0) * 64 + lane, d1n);
        sst(gdm + (kb * 3 + 1) * 64 + lane, d3n);
        sst(gdm + (kb * 3 + 2) * 64 + lane, d4n);
        if (want_res) {  // primal residual: d_new - d_old = u - H z (eq. (14))
          const T zc = zt[k * plane + (lr + M) * EC + (lc + M)];
          const double e1 = (double)d1n - (double)(zc - v1[kk]);
          const double e3 = (double)d3n - (double)(zc - v3[kk]);
          const double e4 = (double)d4n - (double)(zc - v4[kk]);
          rp_acc += e1 * e1 + e3 * e3 + e4 * e4;
        }
        const gptr<T> d2o = gd2 + 2 * (kb * (size_t)(L * 64) + lane);
        // SY: the old d2 and z of this pixel and class, to rebuild Y offset by offset
        [[maybe_unused]] const gptr<const T> d2i = gd2_in + 2 * (kb * (size_t)(L * 64) + lane);
        [[maybe_unused]] const T* zk0 = zt + k * plane + (lr + M) * EC + (lc + M);
        // New d2 = u2 - Y = Y (N - I) and the J^T scatter of c_j (u2 + d2).
        // The h part of offset (dy, dx) lands at (dy, dx + 1) with + and at
        // (dy, dx) with -, the v part at (dy + 1, dx) with + and at (dy, dx)
        // with -.  Walking the destinations (da, db) in row-major order, each
        // one sums its (up to three) terms in registers: the h part of the
        // previous column and the v part of the previous row are carried.
        // Neighbouring lanes reach the same address through different
        // offsets, so the read-modify-writes stay in program order: volatile
        // keeps the compiler from hoisting a later read above an earlier
        // write (LDS executes one wavefront's accesses in order).
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
              T yh, yv;
              if constexpr (SY) {   // Y of this offset again, from z in LDS and the old d2
                const T* zr = zk0 + da * EC + db;
                yh = a.c[jj] * (zr[1] - zr[0]) - d2i[jj * 128];
                yv = a.c[jj] * (zr[EC] - zr[0]) - d2i[jj * 128 + 1];
              } else {
                yh = Y[kk][jj][0];
                yv = Y[kk][jj][1];
              }
              const T nh = yh * m11 + yv * m12;
              const T nv = yh * m12 + yv * m22;
              C2<T> o;
              o.x = nh;
              o.y = nv;
              sst(d2o + jj * 128, o.x);
              sst(d2o + jj * 128 + 1, o.y);
              if (want_res) {  // old d2 = c_j grad z - Y, rebuilt from the LDS tile
                const T* zr = zt + k * plane + (lr + M + da) * EC + (lc + M + db);
                const double oh = (double)(a.c[jj] * (zr[1] - zr[0]) - yh);
                const double ov = (double)(a.c[jj] * (zr[EC] - zr[0]) - yv);
                rp_acc += ((double)nh - oh) * ((double)nh - oh) + ((double)nv - ov) * ((double)nv - ov);
              }
              ah = a.c[jj] * (T(2) * nh + yh);
              av = a.c[jj] * (T(2) * nv + yv);
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
              if constexpr (sizeof(T) == 4 && (M <= 3 || SY)) {
                volatile __attribute__((address_space(3))) T* at =
                    (volatile __attribute__((address_space(3))) T*)(ak + da * EC + db);
                *at = *at + gsum;
              } else {
                // FP64: the LDS atomic add is fast and keeps register pressure down.
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
  if (want_res) {  // fixed-order reduction of the tile's primal-residual partial sums
    double v = rp_acc;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    double* red = reinterpret_cast<double*>(part);
    if (lane == 0) red[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < nw; ++w) t += red[w];
      glob(a.res_tile)[tile] = t;
    }
  }
  const gptr<T> out = glob(a.acc) + (size_t)tile * K * g.ER * g.EC;
  for (int idx = threadIdx.x; idx < K * plane; idx += blockDim.x) {
    const int k = idx / plane;
    const int rem = idx - k * plane;
    const int er = rem / EC, ec = rem - er * EC;
    sst(out + ((size_t)k * g.ER + er) * g.EC + ec, acc[idx]);
  }
}

template <typename T, int M, int KPW, bool VAR, bool PF, bool NT = false>
static hipError_t launch_prox_t(const ProxArgs<T>* descs, int ndesc, int blocks, int threads, size_t lds,
                                hipStream_t st) {
  auto fn = prox_rhs_kernel<T, M, KPW, VAR, PF, NT>;
  static bool lds_set = false;  // idempotent, so a racing second call is harmless
  if (!lds_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kLdsMax);
    if (e != hipSuccess) return e;
    lds_set = true;
  }
  hipLaunchKernelGGL(fn, dim3(blocks), dim3(threads), lds, st, descs, ndesc);
  return hipGetLastError();
}

template <typename T, int M, bool VAR>
static hipError_t launch_prox_m(const ProxArgs<T>* d, int n, int blocks, int threads, int kpw, bool pf, bool nt,
                                size_t lds, hipStream_t st) {
  if (pf) {   // built for the plain FP32 kernel with two classes per wavefront and M <= 2 only
    if constexpr (prox_has_prefetch<T, M, 2, VAR>()) {
      if (kpw == 2) return launch_prox_t<T, M, 2, VAR, true>(d, n, blocks, threads, lds, st);
    }
    return hipErrorInvalidValue;
  }
  if constexpr (!VAR) {   // the streaming build: plain instantiation only
    if (nt) {
      switch (kpw) {
        case 1: return launch_prox_t<T, M, 1, false, false, true>(d, n, blocks, threads, lds, st);
        case 2: return launch_prox_t<T, M, 2, false, false, true>(d, n, blocks, threads, lds, st);
        case 4: return launch_prox_t<T, M, 4, false, false, true>(d, n, blocks, threads, lds, st);
        default: return hipErrorInvalidValue;
      }
    }
  }
  switch (kpw) {
    case 1: return launch_prox_t<T, M, 1, VAR, false>(d, n, blocks, threads, lds, st);
    case 2: return launch_prox_t<T, M, 2, VAR, false>(d, n, blocks, threads, lds, st);
    case 4: return launch_prox_t<T, M, 4, VAR, false>(d, n, blocks, threads, lds, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, bool VAR>
static hipError_t launch_prox_v(const ProxArgs<T>* d, int n, int blocks, int threads, int M, int kpw, bool pf,
                                bool nt, size_t lds, hipStream_t st) {
  switch (M) {
    case 0: return launch_prox_m<T, 0, VAR>(d, n, blocks, threads, kpw, pf, nt, lds, st);
    case 1: return launch_prox_m<T, 1, VAR>(d, n, blocks, threads, kpw, pf, nt, lds, st);
    case 2: return launch_prox_m<T, 2, VAR>(d, n, blocks, threads, kpw, pf, nt, lds, st);
    case 3: return launch_prox_m<T, 3, VAR>(d, n, blocks, threads, kpw, pf, nt, lds, st);
    case 4: return launch_prox_m<T, 4, VAR>(d, n, blocks, threads, kpw, pf, nt, lds, st);
    case 5: return launch_prox_m<T, 5, VAR>(d, n, blocks, threads, kpw, pf, nt, lds, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_prox(const ProxArgs<float>* d, int n, int blocks, int threads, int M, int kpw, bool pf, bool nt,
                       size_t lds, bool variants, hipStream_t st) {
  return variants ? launch_prox_v<float, true>(d, n, blocks, threads, M, kpw, pf, nt, lds, st)
                  : launch_prox_v<float, false>(d, n, blocks, threads, M, kpw, pf, nt, lds, st);
}
hipError_t launch_prox(const ProxArgs<double>* d, int n, int blocks, int threads, int M, int kpw, bool pf, bool nt,
                       size_t lds, bool variants, hipStream_t st) {
  return variants ? launch_prox_v<double, true>(d, n, blocks, threads, M, kpw, pf, nt, lds, st)
                  : launch_prox_v<double, false>(d, n, blocks, threads, M, kpw, pf, nt, lds, st);
}

}  // namespace segsalsa
