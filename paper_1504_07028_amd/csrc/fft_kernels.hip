// z-update of SegSALSA-STR (eq. (12)) as a periodic deconvolution.
//
// G^T G = 3 I + J^T J and, because the periodic shifts P_j are orthogonal,
// J^T J = (sum_j c_j^2) (D_h^T D_h + D_v^T D_v).  The operator is therefore a
// circulant (cyclic convolution, Sec. 4) with the real, even symbol
//     A(ky, kx) = 3 + Wsum (4 sin^2(pi kx / W) + 4 sin^2(pi ky / H)),
// and z = IDFT2[ DFT2(rhs) / A ] for each class image.  Two real class images
// are packed as the real and imaginary parts of one complex image (the symbol
// is real and even, so the two results come back in the real and imaginary
// parts of the inverse transform).
//
// Three passes over HBM per round:
//   rows_fwd : sums the grown-tile partial right-hand sides of the prox
//              kernel (fold), packs class pairs, DFT along rows
//   cols     : DFT along columns, divide by the symbol (and by H W), inverse
//              DFT along columns
//   rows_inv : inverse DFT along rows, unpack into z
// Each 1-D transform runs in LDS as a mixed-radix Stockham FFT (radix 2, 3,
// 4, 5, 8 butterflies in registers; any other prime factor as a direct DFT
// stage).  Twiddles come from exactly rounded tables built once per solve and
// are staged in LDS next to the data.
#include "segsalsa_internal.h"
#include "segsalsa_kernels.h"
#include "fft_math.h"

namespace segsalsa {

// DFT of an odd prime number P of values in registers, using the pairs
// (r, P - r): y_q = a_q + sg i b_q and y_(P-q) = a_q - sg i b_q with
// a_q = v_0 + sum_r (v_r + v_(P-r)) cos(2 pi r q / P) and
// b_q = sum_r (v_r - v_(P-r)) sin(2 pi r q / P), r = 1 .. (P-1)/2.
// cos and sin come from the length-N twiddle table in global memory
// (entry m N / P = exp(-2 pi i m / P)); the index is wavefront-uniform.
template <typename T, int P>
struct BflyOdd {
  __device__ __forceinline__ static void run(C2<T>* v, T sg, gptr<const C2<T>> gtw, int stride) {
    constexpr int Hh = (P - 1) / 2;
    C2<T> sm[Hh], df[Hh];
    C2<T> y0 = v[0];
#pragma unroll
    for (int r = 1; r <= Hh; ++r) {
      sm[r - 1] = cadd(v[r], v[P - r]);
      df[r - 1] = csub(v[r], v[P - r]);
      y0 = cadd(y0, sm[r - 1]);
    }
#pragma unroll
    for (int q = 1; q <= Hh; ++q) {
      C2<T> a = v[0], b = {T(0), T(0)};
#pragma unroll
      for (int r = 1; r <= Hh; ++r) {
        const C2<T> w = ldc(gtw + ((r * q) % P) * stride);
        const T c = w.x, sn = -w.y;
        a.x += sm[r - 1].x * c;
        a.y += sm[r - 1].y * c;
        b.x += df[r - 1].x * sn;
        b.y += df[r - 1].y * sn;
      }
      const C2<T> e = cmuli(b, sg);
      v[q] = cadd(a, e);
      v[P - q] = csub(a, e);
    }
    v[0] = y0;
  }
};

// Odd primes with a register butterfly; larger primes take the direct LDS
// stage (their register butterflies cost more occupancy than they save, as
// measured on the 145-point transforms) or Bluestein.
template <typename T>
__host__ __device__ constexpr bool is_odd_prime_radix(int R) {
  return R == 7 || R == 11 || R == 13;
}

// One Stockham stage with a register butterfly of radix R, in place in LDS.
// nb transforms of length N; element i of transform b sits at b*bs + i*es.
// Ns is the product of the radices of the previous stages.
template <typename T, int R, int EPT, typename TW>
__device__ __forceinline__ void stage_reg(lptr<C2<T>> buf, int N, int nb, int es, int bs, TW tw, gptr<const C2<T>> gtw, int Ns,
                          bool inv) {
  constexpr int IT = (EPT + R - 1) / R;
  const T sg = inv ? T(1) : T(-1);
  const int NR = N / R;
  const int total = nb * NR;
  const int stw = N / (Ns * R);
  const FastDiv fnb(nb), fNR(NR), fNs(Ns);
  C2<T> v[IT][R];
  int ob[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int item = threadIdx.x + it * blockDim.x;
    ob[it] = -1;
    if (item < total) {
      // interleaved transforms (bs == 1): consecutive lanes take consecutive transforms,
      // so one instruction touches one contiguous run of LDS words
      int b, j;
      if (bs == 1) {
        j = (int)fnb.div(item);
        b = item - j * nb;
      } else {
        b = (int)fNR.div(item);
        j = item - b * NR;
      }
      const int k = (int)fNs.mod(j);
      const int base = b * bs;
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = ldc(buf + base + (j + r * NR) * es);
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[it][r] = twmul(v[it][r], ldc(tw + k * r * stw), inv);
      }
      if constexpr (is_odd_prime_radix<T>(R))
        BflyOdd<T, R>::run(v[it], sg, gtw, N / R);
      else
        Bfly<T, R>::run(v[it], sg);
      ob[it] = base + ((j - k) * R + k) * es;
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    if (ob[it] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) stc(buf + ob[it] + r * Ns * es, v[it][r]);
    }
  }
  __syncthreads();
}

// Stockham stage of an odd radix R without a register butterfly, as a
// direct DFT.  The stage computes, for each group j (k = j mod Ns) and output
// q, the sum over r of x_(j + r NR) w_N^(r k stw) w_R^(q r).  The inter-stage
// twiddles w_N^(r k stw) are applied first, once per input element and in
// place (only when Ns > 1; the plans put these radices first); then each
// work item forms the outputs q and R - q from the pre-twiddled inputs,
// pairing the terms r and R - r: with w = w_R^(q r),
//   x_r w + x_(R-r) conj(w) = (x_r + x_(R-r)) Re w + i Im w (x_r - x_(R-r)),
// and output R - q takes conj(w) in place of w, which halves the complex
// multiplies and the LDS reads.
template <typename T, int EPT, typename TW>
__device__ __forceinline__ void stage_generic(lptr<C2<T>> buf, int N, int R, int nb, int es, int bs, TW tw,
                              int Ns, bool inv) {
  const int NR = N / R;
  const int total = nb * N;
  const int stw = N / (Ns * R);
  const FastDiv fnb(nb), fN(N), fNR(NR), fNs(Ns);
  if (Ns > 1) {
    for (int item = threadIdx.x; item < total; item += blockDim.x) {
      int b, rem;
      if (bs == 1) {
        rem = (int)fnb.div(item);
        b = item - rem * nb;
      } else {
        b = (int)fN.div(item);
        rem = item - b * N;
      }
      const int r = (int)fNR.div(rem), j = rem - r * NR;
      const int k = (int)fNs.mod(j);
      if (r > 0 && k > 0) {
        const int idx = b * bs + rem * es;
        stc(buf + idx, twmul(ldc(buf + idx), ldc(tw + r * k * stw), inv));   // r k stw < R Ns stw = N
      }
    }
    __syncthreads();
  }
  // One item per output pair (q, R - q) of a butterfly (q = 0 alone): both
  // outputs take the same pair sums x_r + x_(R-r), x_r - x_(R-r) against
  // conjugate twiddles, so the inputs are read once for two outputs.  R is an
  // odd prime >= 17 here (smaller radices have their own stages), so the
  // nb * N * (R + 1) / (2 R) <= 9/17 nb * N items fit in EPT / 2 + 1 per
  // thread whenever nb * N <= EPT * blockDim.x.
  constexpr int EPTP = EPT / 2 + 1;
  const int half = (R - 1) / 2;
  const int H1 = half + 1;
  const int ptotal = nb * NR * H1;
  const FastDiv fH1(H1), fNRH1(NR * H1);
  C2<T> oa[EPTP], ob[EPTP];
  int ia[EPTP], ib[EPTP];
#pragma unroll
  for (int it = 0; it < EPTP; ++it) {
    const int item = threadIdx.x + it * blockDim.x;
    ia[it] = ib[it] = -1;
    if (item < ptotal) {
      int b, rem;
      if (bs == 1) {
        rem = (int)fnb.div(item);
        b = item - rem * nb;
      } else {
        b = (int)fNRH1.div(item);
        rem = item - b * (NR * H1);
      }
      const int j = (int)fH1.div(rem), q = rem - j * H1;
      const int k = (int)fNs.mod(j);
      const lptr<C2<T>> xj = buf + b * bs + j * es;
      const int sr = NR * es;
      const C2<T> x0 = ldc(xj);
      C2<T> s = x0, t = x0;   // outputs q and R - q
      int m = 0;
      for (int r = 1; r <= half; ++r) {
        m += q;
        if (m >= R) m -= R;
        const C2<T> xa = ldc(xj + r * sr), xb = ldc(xj + (R - r) * sr);
        const C2<T> w = ldc(tw + m * NR);
        const T wi = inv ? -w.y : w.y;
        const T pr = xa.x + xb.x, pi = xa.y + xb.y, dr = xa.x - xb.x, di = xa.y - xb.y;
        s.x += pr * w.x - wi * di;
        s.y += pi * w.x + wi * dr;
        t.x += pr * w.x + wi * di;
        t.y += pi * w.x - wi * dr;
      }
      const int base = b * bs + ((j - k) * R + k) * es;
      oa[it] = s;
      ia[it] = base + q * Ns * es;
      if (q > 0) {
        ob[it] = t;
        ib[it] = base + (R - q) * Ns * es;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < EPTP; ++it) {
    if (ia[it] >= 0) stc(buf + ia[it], oa[it]);
    if (ib[it] >= 0) stc(buf + ib[it], ob[it]);
  }
  __syncthreads();
}


// Mixed-radix Stockham DFT over the given factors (unnormalised).
template <typename T, int EPT, typename TW>
__device__ __forceinline__ void stockham(lptr<C2<T>> buf, int N, int nst, const int* rad, int nb, int es, int bs, TW tw,
                         gptr<const C2<T>> gtw, bool inv) {
  int Ns = 1;
  for (int s = 0; s < nst; ++s) {
    const int R = rad[s];
    switch (R) {
#define SEG_STAGE(RR)                                                                     \
  case RR:                                                                                \
    if constexpr (RR <= 8 || is_odd_prime_radix<T>(RR))                                   \
      stage_reg<T, RR, EPT, TW>(buf, N, nb, es, bs, tw, gtw, Ns, inv);                    \
    else                                                                                  \
      stage_generic<T, EPT, TW>(buf, N, RR, nb, es, bs, tw, Ns, inv);                     \
    break;
      SEG_STAGE(2)
      SEG_STAGE(3)
      SEG_STAGE(4)
      SEG_STAGE(5)
      SEG_STAGE(7)
      SEG_STAGE(8)
      SEG_STAGE(11)
      SEG_STAGE(13)
#undef SEG_STAGE
      default: stage_generic<T, EPT, TW>(buf, N, R, nb, es, bs, tw, Ns, inv); break;
    }
    Ns *= R;
  }
}

// Unnormalised DFT of nb transforms of length p.N in LDS (inv = false:
// exp(-2 pi i ...); inv = true: exp(+2 pi i ...)).  Element i of transform b
// is at buf[b * bs + i * es].  tw: the N twiddles in LDS (Stockham path).
// Bluestein path: X_k = c_k sum_n (x_n c_n) d_(k-n) with c_n = exp(-i pi n^2 / N)
// and d = conj(c), the sum a length-M cyclic convolution by FFT; scr holds
// nb * M elements of LDS scratch.  The workgroup must hold at least
// nb * max(N, M) / EPT threads.
template <typename T, int EPT>
__device__ __forceinline__ void fft_lds(lptr<C2<T>> buf, const FftPlanDev& p, int nb, int es, int bs,
                                        lptr<const C2<T>> tw, const FftTab<T>& tab, lptr<C2<T>> scr, bool inv) {
  if (!p.blu) {
    stockham<T, EPT>(buf, p.N, p.nst, p.rad, nb, es, bs, tw, glob(tab.tw), inv);
    return;
  }
  const int N = p.N, M = p.M;
  const int lgM = __builtin_ctz((unsigned)M);   // M is a power of two
  for (int idx = threadIdx.x; idx < nb * M; idx += blockDim.x) {
    const int b = idx >> lgM, n = idx & (M - 1);
    C2<T> v = {T(0), T(0)};
    if (n < N) {
      C2<T> c = ldc(glob(tab.chirp) + n);
      if (inv) c.y = -c.y;
      v = cmul(ldc(buf + b * bs + n * es), c);
    }
    stc(scr + idx, v);
  }
  __syncthreads();
  stockham<T, EPT>(scr, M, p.mnst, p.mrad, nb, 1, M, glob(tab.twM), glob(tab.twM), false);
  for (int idx = threadIdx.x; idx < nb * M; idx += blockDim.x) {
    const int m = idx & (M - 1);
    C2<T> w;
    if (inv) {  // DFT of conj(d) is conj(DFT(d)) read at -m
      w = ldc(glob(tab.bf) + ((M - m) & (M - 1)));
      w.y = -w.y;
    } else {
      w = ldc(glob(tab.bf) + m);
    }
    stc(scr + idx, cmul(ldc(scr + idx), w));
  }
  __syncthreads();
  stockham<T, EPT>(scr, M, p.mnst, p.mrad, nb, 1, M, glob(tab.twM), glob(tab.twM), true);
  const T invM = T(1) / T(M);
  const FastDiv fN(N);
  for (int idx = threadIdx.x; idx < nb * N; idx += blockDim.x) {
    const int b = (int)fN.div(idx), k = idx - b * N;
    C2<T> c = ldc(glob(tab.chirp) + k);
    if (inv) c.y = -c.y;
    stc(buf + b * bs + k * es, cscale(cmul(ldc(scr + b * M + k), c), invM));
  }
  __syncthreads();
}

// Kernel DFT of the Bluestein convolution: bf = DFT_M(d), d_m = exp(+i pi m^2 / N)
// for m < N and at M - m, zero elsewhere (one workgroup, M elements in LDS).
template <typename T>
__global__ void __launch_bounds__(kFftMaxThreads) bluestein_table_kernel(FftPlanDev p, FftTab<T> tab, C2<T>* bf_out) {
  extern __shared__ __align__(16) unsigned char smem[];
  lptr<C2<T>> buf = (lptr<C2<T>>)smem;
  const int N = p.N, M = p.M;
  for (int m = threadIdx.x; m < M; m += blockDim.x) {
    C2<T> v = {T(0), T(0)};
    const int j = m < N ? m : (M - m < N ? M - m : -1);
    if (j >= 0) {
      v = ldc(glob(tab.chirp) + j);
      v.y = -v.y;
    }
    stc(buf + m, v);
  }
  __syncthreads();
  stockham<T, kFftEptMax>(buf, M, p.mnst, p.mrad, 1, 1, M, glob(tab.twM), glob(tab.twM), false);
  for (int m = threadIdx.x; m < M; m += blockDim.x) bf_out[m] = ldc(buf + m);
}

template <typename T>
hipError_t launch_bluestein_table_t(const FftPlanDev& p, const FftTab<T>& tab, C2<T>* bf_out, hipStream_t st) {
  auto fn = bluestein_table_kernel<T>;
  static bool lds_set = false;
  if (!lds_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kLdsMax);
    if (e != hipSuccess) return e;
    lds_set = true;
  }
  const int threads = p.M / kFftEptMax < 64 ? 64 : (p.M / kFftEptMax > kFftMaxThreads ? kFftMaxThreads : p.M / kFftEptMax);
  hipLaunchKernelGGL(fn, dim3(1), dim3(threads), (size_t)p.M * sizeof(C2<T>), st, p, tab, bf_out);
  return hipGetLastError();
}
hipError_t launch_bluestein_table(const FftPlanDev& p, const FftTab<float>& tab, C2<float>* bf, hipStream_t st) {
  return launch_bluestein_table_t(p, tab, bf, st);
}
hipError_t launch_bluestein_table(const FftPlanDev& p, const FftTab<double>& tab, C2<double>* bf, hipStream_t st) {
  return launch_bluestein_table_t(p, tab, bf, st);
}

template <typename T, int EPT, int MAXT>
__global__ void __launch_bounds__(MAXT) fft_rows_fwd_kernel(const RowFwdArgs<T>* __restrict__ descs, int ndesc) {
  extern __shared__ __align__(16) unsigned char smem[];
  lptr<C2<T>> buf = (lptr<C2<T>>)smem;
  const int blk = xcd_block();   // consecutive rows (neighbouring grown-tile rows) on one XCD
  const RowFwdArgs<T>& a = descs[find_desc(descs, ndesc, blk)];
  const int bid = blk - a.block0;
  const int H = a.g.H, W = a.g.W;
  const int nrb = (H + a.rows_per_block - 1) / a.rows_per_block;
  const int m = bid / nrb;
  const int row0 = (bid - m * nrb) * a.rows_per_block;
  const int nb = min(a.rows_per_block, H - row0);
  const int k0 = 2 * m, k1 = 2 * m + 1;
  lptr<C2<T>> tw = buf + a.rows_per_block * W;  // twiddles, or Bluestein scratch
  const FftTab<T>& tab = a.tab;
  if (!a.plan.blu)
    for (int t = threadIdx.x; t < W; t += blockDim.x) stc(tw + t, ldc(glob(tab.tw) + t));
  // right-hand side (fold_rows): each thread holds at most EPT of the nb * W
  // elements (blockDim.x * EPT >= nb * W, as the LDS FFT needs)
  const bool has1 = k1 < a.K;
  fold_rows<T, EPT>(a, row0, nb, k0, has1, [&](int rr, int c, C2<T> x) { stc(buf + rr * W + c, x); });
  __syncthreads();
  fft_lds<T, EPT>(buf, a.plan, nb, 1, W, tw, tab, tw, false);
  const gptr<C2<T>> out = glob(a.spec) + ((size_t)m * H + row0) * W;
  for (int idx = threadIdx.x; idx < nb * W; idx += blockDim.x) stc(out + idx, ldc(buf + idx));
}

template <typename T, int EPT, int MAXT>
__global__ void __launch_bounds__(MAXT) fft_cols_kernel(const ColArgs<T>* __restrict__ descs, int ndesc) {
  extern __shared__ __align__(16) unsigned char smem[];
  lptr<C2<T>> buf = (lptr<C2<T>>)smem;
  const int blk = xcd_block();   // adjacent column blocks (shared cache lines) on one XCD
  const ColArgs<T>& a = descs[find_desc(descs, ndesc, blk)];
  const int bid = blk - a.block0;
  const int H = a.H, W = a.W;
  const int CB = a.cols_per_block;
  const int ncb = (W + CB - 1) / CB;
  const int m = bid / ncb;
  const int col0 = (bid - m * ncb) * CB;
  const int nb = min(CB, W - col0);
  const FastDiv fnb(nb);
  const gptr<C2<T>> sp = glob(a.spec) + (size_t)m * H * W + col0;
  const FftTab<T>& tab = a.tab;
  lptr<C2<T>> tw = buf + CB * H;  // twiddles, or Bluestein scratch
  if (!a.plan.blu)
    for (int t = threadIdx.x; t < H; t += blockDim.x) stc(tw + t, ldc(glob(tab.tw) + t));
#pragma unroll
  for (int it = 0; it < EPT; ++it) {  // blockDim.x * EPT >= H * nb: loads in flight together
    const int idx = threadIdx.x + it * blockDim.x;
    if (idx < H * nb) {
      const int y = (int)fnb.div(idx), j = idx - y * nb;
      stc(buf + idx, ldc(sp + (size_t)y * W + j));
    }
  }
  __syncthreads();
  // forward column DFT, division by the symbol, inverse column DFT
  fft_lds<T, EPT>(buf, a.plan, nb, nb, 1, tw, tab, tw, false);
  const gptr<const double> sx = glob(a.sx), sy = glob(a.sy);
  for (int idx = threadIdx.x; idx < H * nb; idx += blockDim.x) {
    const int y = (int)fnb.div(idx), j = idx - y * nb;
    const T inv = T(a.scale) / (T(3) + T(a.wsum) * T(sx[col0 + j] + sy[y]));
    stc(buf + idx, cscale(ldc(buf + idx), inv));
  }
  __syncthreads();
  fft_lds<T, EPT>(buf, a.plan, nb, nb, 1, tw, tab, tw, true);
  for (int idx = threadIdx.x; idx < H * nb; idx += blockDim.x) {
    const int y = (int)fnb.div(idx), j = idx - y * nb;
    stc(sp + (size_t)y * W + j, ldc(buf + idx));
  }
}

template <typename T, int EPT, int MAXT>
__global__ void __launch_bounds__(MAXT) fft_rows_inv_kernel(const RowInvArgs<T>* __restrict__ descs, int ndesc) {
  extern __shared__ __align__(16) unsigned char smem[];
  lptr<C2<T>> buf = (lptr<C2<T>>)smem;
  const int blk = xcd_block();
  const RowInvArgs<T>& a = descs[find_desc(descs, ndesc, blk)];
  const int bid = blk - a.block0;
  const int H = a.H, W = a.W;
  const int nrb = (H + a.rows_per_block - 1) / a.rows_per_block;
  const int m = bid / nrb;
  const int row0 = (bid - m * nrb) * a.rows_per_block;
  const int nb = min(a.rows_per_block, H - row0);
  const gptr<const C2<T>> in = glob(a.spec) + ((size_t)m * H + row0) * W;
  const FftTab<T>& tab = a.tab;
  lptr<C2<T>> tw = buf + a.rows_per_block * W;  // twiddles, or Bluestein scratch
  if (!a.plan.blu)
    for (int t = threadIdx.x; t < W; t += blockDim.x) stc(tw + t, ldc(glob(tab.tw) + t));
#pragma unroll
  for (int it = 0; it < EPT; ++it) {  // blockDim.x * EPT >= nb * W: loads in flight together
    const int idx = threadIdx.x + it * blockDim.x;
    if (idx < nb * W) stc(buf + idx, ldc(in + idx));
  }
  __syncthreads();
  fft_lds<T, EPT>(buf, a.plan, nb, 1, W, tw, tab, tw, true);
  const int k0 = 2 * m, k1 = 2 * m + 1;
  const gptr<T> z0 = glob(a.z) + ((size_t)k0 * H + row0) * W;
  const gptr<T> z1 = glob(a.z) + ((size_t)k1 * H + row0) * W;
  const bool has1 = k1 < a.K;
  for (int idx = threadIdx.x; idx < nb * W; idx += blockDim.x) {
    const C2<T> v = ldc(buf + idx);
    z0[idx] = v.x;
    if (has1) z1[idx] = v.y;
  }
}

// One "LDS limit raised" flag per kernel instantiation (FN is the kernel).
template <auto FN, typename A>
static hipError_t launch_fft(const A* descs, int ndesc, int blocks, int threads, size_t lds, hipStream_t st) {
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

template <auto F2, auto F4, auto F8, auto F16, typename A>
static hipError_t launch_ept(int ept, const A* d, int n, int blocks, int threads, size_t lds, hipStream_t st) {
  switch (ept) {
    case 2: return launch_fft<F2>(d, n, blocks, threads, lds, st);
    case 4: return launch_fft<F4>(d, n, blocks, threads, lds, st);
    case 8: return launch_fft<F8>(d, n, blocks, threads, lds, st);
    case 16: return launch_fft<F16>(d, n, blocks, threads, lds, st);
    default: return hipErrorInvalidValue;
  }
}

#define SEG_FFT_LAUNCHER(NAME, ARGS, KERNEL)                                                                       \
  hipError_t NAME(const ARGS<float>* d, int n, int blocks, int ept, int threads, bool, size_t lds, hipStream_t st) { \
    return launch_ept<KERNEL<float, 2, kFftMaxThreads>, KERNEL<float, 4, kFftMaxThreads>,                           \
                      KERNEL<float, 8, kFftMaxThreads>, KERNEL<float, 16, kFftMaxThreads>>(ept, d, n, blocks,       \
                                                                                            threads, lds, st);      \
  }                                                                                                                 \
  hipError_t NAME(const ARGS<double>* d, int n, int blocks, int ept, int threads, bool narrow, size_t lds,           \
                  hipStream_t st) {                                                                                 \
    if (narrow) {                                                                                                   \
      if (threads > kFftNarrowThreads) return hipErrorInvalidValue;                                                 \
      return launch_ept<KERNEL<double, 2, kFftNarrowThreads>, KERNEL<double, 4, kFftNarrowThreads>,                 \
                        KERNEL<double, 8, kFftNarrowThreads>, KERNEL<double, 16, kFftNarrowThreads>>(               \
          ept, d, n, blocks, threads, lds, st);                                                                     \
    }                                                                                                               \
    return launch_ept<KERNEL<double, 2, kFftMaxThreads>, KERNEL<double, 4, kFftMaxThreads>,                         \
                      KERNEL<double, 8, kFftMaxThreads>, KERNEL<double, 16, kFftMaxThreads>>(ept, d, n, blocks,     \
                                                                                              threads, lds, st);    \
  }

SEG_FFT_LAUNCHER(launch_rows_fwd, RowFwdArgs, fft_rows_fwd_kernel)
SEG_FFT_LAUNCHER(launch_cols, ColArgs, fft_cols_kernel)
SEG_FFT_LAUNCHER(launch_rows_inv, RowInvArgs, fft_rows_inv_kernel)
#undef SEG_FFT_LAUNCHER

}  // namespace segsalsa
