// Kernel launchers of the SegSALSA-STR library (defined in the .hip files).
#pragma once

#include "segsalsa_internal.h"

namespace segsalsa {

// Patches of 9x9 and larger rebuild Y = J z - d2 in the prox kernel's update
// phase instead of keeping it in registers.
template <int M>
__host__ __device__ constexpr bool prox_streams_y() {
  return M >= 4;
}

// Largest workgroup the prox kernel instantiation <T, M, KPW> is compiled for:
// each lane keeps KPW classes x 2L entries of the J-split block in registers,
// so the wavefronts per SIMD (and hence per workgroup) shrink as L grows.
template <typename T, int M, int KPW, bool PF = false>
__host__ __device__ constexpr int prox_max_threads() {
  constexpr int L = (2 * M + 1) * (2 * M + 1);
  // registers held per class: Y's 2L values, or (patches of 9x9 and larger,
  // which rebuild Y in the update phase) the carries of the scatter
  constexpr int LY = prox_streams_y<M>() ? 2 * M + 2 : L;
  constexpr int vg = (PF ? 2 : 1) * KPW * 2 * LY * (int)(sizeof(T) / 4) + (PF ? 56 : 48);
  constexpr int wps = 512 / vg;
  constexpr int w = wps >= 4 ? 4 : (wps < 1 ? 1 : wps);
  return w * 4 * 64;
}

// The prefetching build of the prox kernel exists for the plain FP32 kernel
// with two classes per wavefront and patches up to 5x5.
template <typename T, int M, int KPW, bool VAR>
__host__ __device__ constexpr bool prox_has_prefetch() {
  return sizeof(T) == 4 && KPW == 2 && M <= 2 && !VAR;
}
inline bool prox_has_prefetch_rt(bool fp64, int M, int kpw) { return !fp64 && kpw == 2 && M <= 2; }

inline int prox_max_threads_rt(bool fp64, int M, int kpw, bool pf = false) {
#define SEG_CASE(MM)                                                                                         \
  case MM:                                                                                                   \
    if (fp64) return kpw == 1 ? prox_max_threads<double, MM, 1>() : kpw == 2 ? prox_max_threads<double, MM, 2>() \
                                                                           : prox_max_threads<double, MM, 4>(); \
    if (pf) return prox_max_threads<float, MM, 2, true>();                                                   \
    return kpw == 1 ? prox_max_threads<float, MM, 1>() : kpw == 2 ? prox_max_threads<float, MM, 2>()           \
                                                                 : prox_max_threads<float, MM, 4>();
  switch (M) {
    SEG_CASE(0)
    SEG_CASE(1)
    SEG_CASE(2)
    SEG_CASE(3)
    SEG_CASE(4)
    SEG_CASE(5)
    default: return 0;
  }
#undef SEG_CASE
}

// Per-round launches over a table of per-image descriptors in device memory.
// variants: the instantiation with the general Schatten p, the simplex g4 and the
// primal-residual accumulation compiled in (required for descriptors with res_tile set)
// pf: the prefetching build (prox_has_prefetch; only without variants)
// nt: the streaming build (nontemporal state accesses; only without variants
// or prefetch, ignored otherwise)
hipError_t launch_prox(const ProxArgs<float>* d, int n, int blocks, int threads, int M, int kpw, bool pf, bool nt,
                       size_t lds, bool variants, hipStream_t st);
hipError_t launch_prox(const ProxArgs<double>* d, int n, int blocks, int threads, int M, int kpw, bool pf, bool nt,
                       size_t lds, bool variants, hipStream_t st);

// FFT passes; narrow (FP64 only): the instantiation built for at most 512
// threads per workgroup (threads must not exceed it)
hipError_t launch_rows_fwd(const RowFwdArgs<float>* d, int n, int blocks, int ept, int threads, bool narrow, size_t lds,
                           hipStream_t st);
hipError_t launch_rows_fwd(const RowFwdArgs<double>* d, int n, int blocks, int ept, int threads, bool narrow, size_t lds,
                           hipStream_t st);
hipError_t launch_cols(const ColArgs<float>* d, int n, int blocks, int ept, int threads, bool narrow, size_t lds,
                           hipStream_t st);
hipError_t launch_cols(const ColArgs<double>* d, int n, int blocks, int ept, int threads, bool narrow, size_t lds,
                           hipStream_t st);
hipError_t launch_rows_inv(const RowInvArgs<float>* d, int n, int blocks, int ept, int threads, bool narrow, size_t lds,
                           hipStream_t st);
hipError_t launch_rows_inv(const RowInvArgs<double>* d, int n, int blocks, int ept, int threads, bool narrow, size_t lds,
                           hipStream_t st);

// FFT passes for power-of-two lengths N in 64 .. 4096 (fft_pow2_kernels.hip):
// N / 16 threads per transform, so threads = (rows or columns per block) * N / 16.
hipError_t launch_rows_fwd_p2(const RowFwdArgs<float>* d, int n, int blocks, int N, int threads, size_t lds,
                              hipStream_t st);
hipError_t launch_rows_fwd_p2(const RowFwdArgs<double>* d, int n, int blocks, int N, int threads, size_t lds,
                              hipStream_t st);
hipError_t launch_cols_p2(const ColArgs<float>* d, int n, int blocks, int N, int threads, size_t lds, hipStream_t st);
hipError_t launch_cols_p2(const ColArgs<double>* d, int n, int blocks, int N, int threads, size_t lds, hipStream_t st);
hipError_t launch_rows_inv_p2(const RowInvArgs<float>* d, int n, int blocks, int N, int threads, size_t lds,
                              hipStream_t st);
hipError_t launch_rows_inv_p2(const RowInvArgs<double>* d, int n, int blocks, int N, int threads, size_t lds,
                              hipStream_t st);
// FFT passes for sides that take Bluestein's transform, with the two
// length-MM convolution FFTs (MM in 64 .. 4096) on the same engine
// (fft_blu_kernels.hip): threads = (rows or columns per block) * MM / 16.
hipError_t launch_rows_fwd_blu(const RowFwdArgs<float>* d, int n, int blocks, int MM, int threads, size_t lds,
                               hipStream_t st);
hipError_t launch_rows_fwd_blu(const RowFwdArgs<double>* d, int n, int blocks, int MM, int threads, size_t lds,
                               hipStream_t st);
hipError_t launch_cols_blu(const ColArgs<float>* d, int n, int blocks, int MM, int threads, size_t lds, hipStream_t st);
hipError_t launch_cols_blu(const ColArgs<double>* d, int n, int blocks, int MM, int threads, size_t lds, hipStream_t st);
hipError_t launch_rows_inv_blu(const RowInvArgs<float>* d, int n, int blocks, int MM, int threads, size_t lds,
                               hipStream_t st);
hipError_t launch_rows_inv_blu(const RowInvArgs<double>* d, int n, int blocks, int MM, int threads, size_t lds,
                               hipStream_t st);
// Column pass by the periodic tridiagonal recursions (tri_kernels.hip): lpt
// rows per thread (16 or 32), at least cols_per_block * ceil(H / lpt) threads,
// tri_lds(threads, element size) bytes of LDS.
hipError_t launch_cols_tri(const ColArgs<float>* d, int n, int blocks, int lpt, int threads, size_t lds,
                           hipStream_t st);
hipError_t launch_cols_tri(const ColArgs<double>* d, int n, int blocks, int lpt, int threads, size_t lds,
                           hipStream_t st);
inline size_t tri_lds(int threads, size_t ts) { return ((2 * (size_t)threads * ts + 15) & ~size_t(15)) + 4 * (size_t)threads * ts; }
constexpr int kP2Min = 64, kP2Max = 4096;
inline bool p2_length(int n) { return n >= kP2Min && n <= kP2Max && (n & (n - 1)) == 0; }
// LDS elements per transform of the power-of-two kernels (one pad element every 16, plus one)
inline size_t p2_region(int n) { return (size_t)n + n / 16 + 1; }

// Set-up, initialisation and data-movement kernels (misc_kernels.hip).
template <typename T>
struct SetupArgs {
  TileGeom g;
  int* frow;    // [kFoldStride][H]
  int* fcol;    // [kFoldStride][W]
  int H, W;
  C2<T>* twW;   // exp(-2 pi i t / W), t < W
  C2<T>* twH;   // exp(-2 pi i t / H), t < H
  double* sx;   // 4 sin^2(pi t / W)
  double* sy;   // 4 sin^2(pi t / H)
  int MW, MH;   // Bluestein convolution lengths (0: not used)
  C2<T>* chW;   // exp(-i pi t^2 / W), t < W (Bluestein)
  C2<T>* chH;
  C2<T>* twMW;  // exp(-2 pi i t / MW), t < MW
  C2<T>* twMH;
};
hipError_t launch_bluestein_table(const FftPlanDev& p, const FftTab<float>& tab, C2<float>* bf, hipStream_t st);
hipError_t launch_bluestein_table(const FftPlanDev& p, const FftTab<double>& tab, C2<double>* bf, hipStream_t st);
hipError_t launch_setup(const SetupArgs<float>& a, hipStream_t st);
hipError_t launch_setup(const SetupArgs<double>& a, hipStream_t st);

template <typename T>
struct InitArgs {
  TileGeom g;
  int K;
  int is_logits;
  const T* input;   // [K][H][W]
  T* z;             // [K][H][W]
  T* phat;          // tile layout
  T* dm;            // tile layout
  int* flags;
};
hipError_t launch_init(const InitArgs<float>& a, hipStream_t st);
hipError_t launch_init(const InitArgs<double>& a, hipStream_t st);

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st);
// Copy n host bytes into device memory through kernel arguments (no host
// staging buffer has to outlive the call; capturable in a graph).
hipError_t launch_store(void* dst, const void* src, size_t n, hipStream_t st);
// Two such stores of at most kStorePairMax bytes each in one launch.
constexpr int kStorePairMax = 64;
hipError_t launch_store_pair(void* dst0, const void* src0, size_t n0, void* dst1, const void* src1, size_t n1,
                             hipStream_t st);

// Conversion between the tile layout and canonical class-planar arrays.
template <typename T>
struct StateArgs {
  TileGeom g;
  int K, L;
  int to_canonical;   // 1: tile -> canonical, 0: canonical -> tile
  T* phat_t; T* dm_t; T* d2_t;                      // tile layout (workspace)
  T* phat; T* d1; T* d2; T* d3; T* d4;              // canonical (may be null)
};
hipError_t launch_state(const StateArgs<float>& a, hipStream_t st);
hipError_t launch_state(const StateArgs<double>& a, hipStream_t st);

// Convergence diagnostics (residual_kernels.hip).
constexpr int kDiagBlocks = 1024;
template <typename T>
struct DiagArgs {
  TileGeom g;
  int K;
  int pkind;
  double pval;
  double lambda, wsum;
  const T* z;        // [K][H][W] current z
  T* zprev;          // [K][H][W] z before the round; scratch for the projection in the objective
  const T* phat;     // tile layout
  double* partial;   // per-block partial sums
  double* out;       // [0] primal^2, [1] dual^2 / mu^2, [2] objective
  double cw[kMaxL];  // multipliers c_j
};
hipError_t launch_copy(const float* src, float* dst, size_t n, hipStream_t st);
hipError_t launch_copy(const double* src, double* dst, size_t n, hipStream_t st);
hipError_t launch_dual_res(const DiagArgs<float>& a, hipStream_t st);
hipError_t launch_dual_res(const DiagArgs<double>& a, hipStream_t st);
hipError_t launch_objective(const DiagArgs<float>& a, hipStream_t st);
hipError_t launch_objective(const DiagArgs<double>& a, hipStream_t st);
hipError_t launch_reduce(const double* partial, int count, double* out, int slot, hipStream_t st);

hipError_t launch_labels(int K, int H, int W, const float* z, int32_t* labels, hipStream_t st);
hipError_t launch_labels(int K, int H, int W, const double* z, int32_t* labels, hipStream_t st);

// Reverse sweep (adjoint_kernels.hip).  The adjoint kernel keeps, per lane,
// KPW classes x 2L entries of the J-split block and L FP64 partial sums of
// the multiplier cotangents; the per-lane register estimate below follows
// the compiler's allocation for M <= 2 (about 6 (FP32) or 8 (FP64) VGPRs per
// offset and class over a base of ~130), so that the launch bound does not
// force spills.
template <typename T, int M, int KPW>
__host__ __device__ constexpr int adj_max_threads() {
  constexpr int L = (2 * M + 1) * (2 * M + 1);
  constexpr int vg = sizeof(T) == 4 ? 128 + KPW * (6 * L + 4) : 136 + KPW * (8 * L + 6);
  constexpr int wps = 512 / vg;
  constexpr int w = wps >= 4 ? 4 : (wps < 1 ? 1 : wps);
  return w * 4 * 64;
}

// Waves per SIMD the adjoint kernel is compiled for: FP32 with one class per
// wavefront and M <= 1 fits 128 VGPRs (two 8-wave workgroups per compute
// unit, so one runs its FP64 closed forms while the other streams); the
// others keep the register budget of a single workgroup.
template <typename T, int M, int KPW>
__host__ __device__ constexpr int adj_min_waves() {
  return sizeof(T) == 4 && M <= 1 && KPW == 1 ? 4 : 1;
}

inline int adj_max_threads_rt(bool fp64, int M, int kpw) {
#define SEG_CASE(MM)                                                                                       \
  case MM:                                                                                                 \
    if (fp64) return kpw == 1 ? adj_max_threads<double, MM, 1>() : kpw == 2 ? adj_max_threads<double, MM, 2>() \
                                                                          : adj_max_threads<double, MM, 4>(); \
    return kpw == 1 ? adj_max_threads<float, MM, 1>() : kpw == 2 ? adj_max_threads<float, MM, 2>()           \
                                                                : adj_max_threads<float, MM, 4>();
  switch (M) {
    SEG_CASE(0)
    SEG_CASE(1)
    SEG_CASE(2)
    SEG_CASE(3)
    SEG_CASE(4)
    SEG_CASE(5)
    default: return 0;
  }
#undef SEG_CASE
}

template <typename T>
struct AdjArgs {
  TileGeom g;
  int K, nw;
  const T* __restrict__ z;     // [K][H][W] z before the round
  const T* __restrict__ zn;    // [K][H][W] z after the round
  const T* __restrict__ r;     // [K][H][W] A^{-1} applied to the cotangent of zn
  const T* __restrict__ phat;  // tile layout
  const T* __restrict__ dm;    // multipliers before the round (tile layout)
  const T* __restrict__ d2;
  T* __restrict__ bdm;         // their cotangents: in, after the round; out, before it
  T* __restrict__ bd2;
  T* __restrict__ pbar;        // tile layout, accumulated cotangent of p_hat (data term)
  T* __restrict__ acc;         // [tile][K][ER][EC] partial sums of the cotangent of z
  double* __restrict__ gpart;  // [tile][L + 2] running totals: c_j, lambda * mu, <D rb, D zn>
  double mu, tau;
  int pkind;
  T c[kMaxL];
};

template <typename T>
struct AdjIOArgs {
  TileGeom g;
  int K, is_logits;
  const T* grad_z;     // [K][H][W]
  const T* input;      // [K][H][W]
  const T* phat;       // tile layout
  const T* pbar;       // tile layout
  T* acc;              // grown-tile partial sums
  const int* frow;
  const int* fcol;
  T* grad_input;       // [K][H][W]
};

struct AdjParamOut {
  double* tot;           // [L + 2] device scratch
  double* grad_weights;  // [L] device, may be null
  double* grad_lambda;   // [1] device, may be null
  double mu;
  double c[kMaxL];       // multipliers as applied (rounded to the element type)
};

hipError_t launch_adj_prox(const AdjArgs<float>& a, int blocks, int threads, int M, int kpw, size_t lds,
                           hipStream_t st);
hipError_t launch_adj_prox(const AdjArgs<double>& a, int blocks, int threads, int M, int kpw, size_t lds,
                           hipStream_t st);
hipError_t launch_adj_load(const AdjIOArgs<float>& a, hipStream_t st);
hipError_t launch_adj_load(const AdjIOArgs<double>& a, hipStream_t st);
hipError_t launch_adj_input(const AdjIOArgs<float>& a, hipStream_t st);
hipError_t launch_adj_input(const AdjIOArgs<double>& a, hipStream_t st);
hipError_t launch_adj_params(const double* gpart, int ntiles, int L, const AdjParamOut& o, hipStream_t st);
hipError_t launch_copy_bytes(void* dst, const void* src, size_t bytes, hipStream_t st);
// bytes: a multiple of 16; both pointers 16-byte aligned
hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t st);

}  // namespace segsalsa
