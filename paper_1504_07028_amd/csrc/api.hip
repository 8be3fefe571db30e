// Host runtime of the SegSALSA-STR C ABI: argument validation, plan (tile
// grid, FFT factorisations, workspace layout) and the per-round launch
// sequence.  See include/segsalsa.h for the contract of each entry point.
#include "segsalsa.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "segsalsa_internal.h"
#include "segsalsa_kernels.h"

using namespace segsalsa;

// Workspace of segsalsa_str_solve_noalloc: one array per GPU, held until the
// process ends.  In host code `scratch` only names the symbol; its device
// address on the current GPU comes from hipGetSymbolAddress (noalloc_scratch).
static __device__ __align__(256) unsigned char scratch[SEGSALSA_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_last_error;

segsalsa_status fail(segsalsa_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

segsalsa_status hip_fail(hipError_t e, const char* what) {
  return fail(SEGSALSA_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
// Dynamic LDS one workgroup may use (gfx950 has 160 KiB per CU).
constexpr size_t kLdsBudget = 160 * 1024;
// Per-round prox state above which its accesses bypass the caches: measured,
// the streaming build is 5-11 % faster at 2048x2048 (29 GB) and on the
// 64-image batch (9.5 GB), 8 % at 610x340 FP64 (1.6 GB), within 1 % at
// 610x340 FP32 (0.8 GB), and 9-25 % slower at 145x145 (0.15-0.29 GB), whose
// state the 256 MB MALL keeps from round to round.
constexpr size_t kStreamBytes = size_t(1) << 30;

// Factor a length into radices: primes above 13 (direct DFT stages) first,
// so they run with Ns = 1 and need no inter-stage twiddles, then 8s, 4 and
// 2, 3s, 5s, and the other primes in increasing order.
int factorize(int N, int* rad) {
  std::vector<int> r;
  int n = N;
  while (n % 8 == 0) { r.push_back(8); n /= 8; }
  if (n % 4 == 0) { r.push_back(4); n /= 4; }
  if (n % 2 == 0) { r.push_back(2); n /= 2; }
  while (n % 3 == 0) { r.push_back(3); n /= 3; }
  while (n % 5 == 0) { r.push_back(5); n /= 5; }
  for (int f = 7; (long long)f * f <= n; f += 2)
    while (n % f == 0) { r.push_back(f); n /= f; }
  if (n > 1) r.push_back(n);
  std::stable_partition(r.begin(), r.end(), [](int f) { return f > 13; });
  for (size_t i = 0; i < r.size(); ++i) rad[i] = r[i];
  return (int)r.size();
}

// Largest prime factor handled by a direct DFT stage; longer primes go
// through Bluestein (SEGSALSA_BLUESTEIN_PRIME overrides, for tuning).  The
// paired direct stage costs (R - 1) / 2 complex updates per output; a
// Bluestein transform costs two power-of-two transforms of length >= 2N - 1:
// measured, a direct 61-point stage runs the 610-long columns in half the
// time of Bluestein (length 2048).
int bluestein_prime() {
  static int v = -1;
  if (v < 0) {
    const char* e = std::getenv("SEGSALSA_BLUESTEIN_PRIME");
    v = e ? std::max(5, std::atoi(e)) : 100;
  }
  return v;
}

FftPlanDev make_fft_plan(int N) {
  FftPlanDev p;
  std::memset(&p, 0, sizeof(p));
  p.N = N;
  p.nst = factorize(N, p.rad);
  int big = 1;
  for (int i = 0; i < p.nst; ++i) big = std::max(big, p.rad[i]);
  if (big > bluestein_prime() && big != 8) {
    int M = 1;
    while (M < 2 * N - 1) M *= 2;
    p.blu = 1;
    p.M = M;
    p.mnst = factorize(M, p.mrad);
  }
  return p;
}

constexpr int kTriThreads = 512;   // workgroup size of the tridiagonal column pass (see plan_with)
constexpr double kTriMinGap = 0.1;  // smallest 1 - rho of an FP32 solve by the recursions (see plan_with)

// Lengths the fixed-structure engine runs: powers of two 64 .. 4096, and
// lengths taking Bluestein whose convolution length is in that range.
bool engine_length(int n) {
  const FftPlanDev f = make_fft_plan(n);
  return f.blu ? p2_length(f.M) : p2_length(n);
}

struct Plan {
  bool fp64;
  size_t ts;     // sizeof(T)
  int K, H, W, M, L, P;
  TileGeom g;
  int nw, kpw;   // prox workgroup: wavefronts and classes per wavefront
  bool pf;       // the prefetching build of the prox kernel
  size_t prox_lds;
  int anw, akpw;  // adjoint workgroup (differentiable solves only)
  int g4s;        // simplex g4: the prox kernel stages v4 of all classes in LDS
  size_t adj_lds;
  FftPlanDev frow, fcol;
  // FFT workgroups: transforms per workgroup, threads, elements per thread
  int rows_per_block, row_threads, row_ept;
  int row_p2, col_p2;   // length of the fixed-structure row (column) engine, 0: general kernels
  bool row_blu, col_blu;   // the engine runs the Bluestein convolution (its length is frow.M / fcol.M)
  bool col_tri;            // the column pass by the tridiagonal recursions (col_ept rows per thread)
  size_t row_lds;
  int cols_per_block, col_threads, col_ept;
  size_t col_lds;
  bool tuned;     // the prox tile, classes per wavefront and FFT blocking came from the tuning table
  // workspace offsets (bytes)
  size_t off_flags, off_twW, off_twH, off_sx, off_sy, off_frow, off_fcol, off_phat, off_dm, off_d2, off_acc, off_spec,
      off_zprev, off_restile, off_partial, off_out, off_chW, off_chH, off_bfW, off_bfH, off_twMW, off_twMH, total;
  int npartial;
};

int ceil_div(int a, int b) { return (a + b - 1) / b; }

constexpr int kTargetGroups = 256;   // one workgroup per compute unit of an MI355X

TileGeom tile_geom(const Plan& p, int tr, int tc) {
  TileGeom g;
  g.H = p.H; g.W = p.W; g.M = p.M;
  g.ntr = ceil_div(p.H, std::min(tr, p.H));
  g.ntc = ceil_div(p.W, std::min(tc, p.W));
  g.TR = ceil_div(p.H, g.ntr);
  g.TC = ceil_div(p.W, g.ntc);
  g.ER = g.TR + 2 * p.M + 1;
  g.EC = g.TC + 2 * p.M + 1;
  g.steps = ceil_div(g.TR * g.TC, 64);
  return g;
}

bool fold_lists_fit(const TileGeom& g) {
  for (int r = 0; r < g.H; ++r)
    if (fold_list(g, r, true, nullptr, 0) < 0) return false;
  for (int c = 0; c < g.W; ++c)
    if (fold_list(g, c, false, nullptr, 0) < 0) return false;
  return true;
}

// Tile columns the vector fold handles (fold_gather_vec): one width, a
// multiple of kFoldVec elements, at least 2M + 2.
bool vector_fold_fits(const TileGeom& g, size_t ts) {
  return g.W % g.ntc == 0 && g.TC % (int)(16 / ts) == 0 && g.TC >= 2 * g.M + 2;
}

// LDS bytes of the prox workgroup (and of the reverse sweep's, for
// differentiable solves) on the grown tile of g.
size_t prox_lds_fwd(const Plan& p, const TileGeom& g) {
  // partial sums [2][6][nw][64] (T), per-pixel FP64 sums [6][64] and coefficients [5][64], v4 stage (simplex g4)
  const size_t part = 12 * (size_t)p.nw * 64 + (p.g4s ? 2 * (size_t)p.K * 64 : 0);
  return (2 * (size_t)p.K * g.ER * g.EC + part) * p.ts + 11 * 64 * 8 + 16;
}
size_t prox_lds_adj(const Plan& p, const TileGeom& g) {
  // reverse sweep: z, the solved cotangent and the accumulator over the grown tile
  return p.anw ? (3 * (size_t)p.K * g.ER * g.EC + 20 * (size_t)p.anw * 64) * p.ts + 20 * 64 * 8 + 16 : 0;
}

// Tile shapes that fit LDS, best first by the cost model: a workgroup
// processes one tile in ceil(pixels / 64) steps plus a fixed load/store
// phase and tiles run in batches of (compute units x resident workgroups),
// so the cost is batches x (steps + 1); ties go to shapes whose tile columns
// allow the vector fold (one width, a multiple of 16 bytes of elements, at
// least 2M + 2), then to the smaller grown-tile overhead.
std::vector<TileGeom> tile_candidates(const Plan& p) {
  static const int rows[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32};
  static const int cols[] = {8, 12, 16, 20, 24, 32, 40, 48, 64, 96, 128};
  // resident workgroups per CU allowed by the register budget of the chosen instantiation
  const int waves_per_simd = std::max(1, prox_max_threads_rt(p.fp64, p.M, p.kpw, p.pf) / 256);
  const int occ_regs = std::max(1, (4 * waves_per_simd) / p.nw);
  struct Cand {
    TileGeom g;
    double cost;
    bool vf;
    double over;
  };
  std::vector<Cand> cs;
  for (int tr : rows) {
    for (int tc : cols) {
      TileGeom g = tile_geom(p, tr, tc);
      bool dup = false;
      for (const Cand& c : cs) dup |= c.g.ntr == g.ntr && c.g.ntc == g.ntc;
      if (dup) continue;
      const size_t lds = std::max(prox_lds_fwd(p, g), prox_lds_adj(p, g));
      if (lds > kLdsBudget) continue;
      const int occ = std::max(1, std::min(occ_regs, (int)(kLdsBudget / lds)));
      const long long slots = (long long)kTargetGroups * occ;
      const long long batches = (g.ntiles() + slots - 1) / slots;
      cs.push_back({g, (double)batches * (g.steps + 1), vector_fold_fits(g, p.ts),
                    (double)g.ER * g.EC / ((double)g.TR * g.TC)});
    }
  }
  std::stable_sort(cs.begin(), cs.end(), [](const Cand& a, const Cand& b) {
    if (a.cost != b.cost) return a.cost < b.cost;
    if (a.vf != b.vf) return a.vf;
    return a.over < b.over;
  });
  std::vector<TileGeom> out;
  for (const Cand& c : cs) out.push_back(c.g);
  return out;
}

// Tile grid of the prox kernel: force_r x force_c (a tuned shape) if it fits,
// else the best candidate whose fold lists fit.
bool choose_tiles(Plan& p, int force_r, int force_c) {
  auto take = [&](const TileGeom& g) {
    p.g = g;
    p.prox_lds = prox_lds_fwd(p, g);
    p.adj_lds = prox_lds_adj(p, g);
  };
  if (force_r > 0 && force_c > 0) {
    TileGeom g = tile_geom(p, force_r, force_c);
    if (std::max(prox_lds_fwd(p, g), prox_lds_adj(p, g)) > kLdsBudget || !fold_lists_fit(g)) return false;
    take(g);
    return true;
  }
  for (const TileGeom& g : tile_candidates(p)) {
    if (!fold_lists_fit(g)) continue;
    take(g);
    return true;
  }
  return false;
}

// Elements per thread of an LDS FFT workgroup of `threads` threads holding
// `items` complex elements: the fewest of 2, 4, 8, 16 with threads * ept >=
// items, or 0 if even 16 do not suffice.
int fft_ept(long long items, int threads) {
  for (int e = 2; e <= kFftEptMax; e *= 2)
    if ((long long)threads * e >= items) return e;
  return 0;
}

// Threads for `items` elements at about `per` elements per thread (a
// multiple of 64, at most 1024).
int fft_threads_for(long long items, int per) {
  long long t = (items + per - 1) / per;
  t = (t + 63) / 64 * 64;
  return (int)std::max<long long>(64, std::min<long long>(t, kFftMaxThreads));
}

// ---------------------------------------------------------------------------
// Tuning table: launch shapes for images of one (K, H, W, M, precision),
// measured by segsalsa_str_autotune or set by the caller, read by the planner.
// ---------------------------------------------------------------------------
struct TuneKey {
  int K, H, W, M, fp64;
  bool operator<(const TuneKey& o) const {
    return std::tie(K, H, W, M, fp64) < std::tie(o.K, o.H, o.W, o.M, o.fp64);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, segsalsa_tuning> g_tune;

bool tuning_lookup(int K, int H, int W, int M, bool fp64, segsalsa_tuning& out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(TuneKey{K, H, W, M, fp64 ? 1 : 0});
  if (it == g_tune.end()) return false;
  out = it->second;
  return true;
}

// ---------------------------------------------------------------------------
// Validation
// ---------------------------------------------------------------------------

// Parameters shared by every image of a solve.
struct Common {
  bool fp64;
  size_t ts;
  int M, L, pkind;
  double w[kMaxL];
  double p;
  int iters, logits, every, warm, graph;
  double tol;
  int g4s = 0;    // g4 as the probability-simplex projection
  int grad = 0;   // plan for the reverse sweep as well (tiles sized for its LDS)
};

segsalsa_status validate_common(int M, const double* weights, double p, int iters, int logits, int every, double tol,
                                int warm, int graph, int g4s, segsalsa_precision prec, Common& c) {
  if (prec != SEGSALSA_FP32 && prec != SEGSALSA_FP64) return fail(SEGSALSA_ERR_INVALID_ARG, "bad precision %d", (int)prec);
  if (M < 0) return fail(SEGSALSA_ERR_INVALID_ARG, "patch_radius = %d < 0", M);
  if (M > kMaxM) return fail(SEGSALSA_ERR_UNSUPPORTED, "patch_radius = %d > %d", M, kMaxM);
  if (!weights) return fail(SEGSALSA_ERR_INVALID_ARG, "patch_weights is NULL");
  const int L = (2 * M + 1) * (2 * M + 1);
  for (int j = 0; j < L; ++j)
    if (!std::isfinite(weights[j])) return fail(SEGSALSA_ERR_INVALID_ARG, "patch weight %d not finite", j);
  if (std::isnan(p)) return fail(SEGSALSA_ERR_INVALID_ARG, "schatten_p is NaN");
  if (!(p >= 1.0)) return fail(SEGSALSA_ERR_INVALID_ARG, "schatten_p = %g < 1 is not a norm", p);
  if (iters < 0) return fail(SEGSALSA_ERR_INVALID_ARG, "iters = %d < 0", iters);
  if (logits != 0 && logits != 1) return fail(SEGSALSA_ERR_INVALID_ARG, "input_is_logits = %d", logits);
  if (every < 0) return fail(SEGSALSA_ERR_INVALID_ARG, "residual_every = %d", every);
  if (!std::isfinite(tol) || tol < 0.0) return fail(SEGSALSA_ERR_INVALID_ARG, "tol = %g", tol);
  if (tol > 0.0 && every == 0) return fail(SEGSALSA_ERR_INVALID_ARG, "tol > 0 needs residual_every > 0");
  if (warm != 0 && warm != 1) return fail(SEGSALSA_ERR_INVALID_ARG, "warm_start = %d", warm);
  if (graph != 0 && graph != 1) return fail(SEGSALSA_ERR_INVALID_ARG, "use_graph = %d", graph);
  if (graph && every > 0) return fail(SEGSALSA_ERR_INVALID_ARG, "use_graph cannot be combined with residual_every");
  if (g4s != 0 && g4s != 1) return fail(SEGSALSA_ERR_INVALID_ARG, "g4_simplex = %d", g4s);
  c.fp64 = prec == SEGSALSA_FP64;
  c.ts = c.fp64 ? 8 : 4;
  c.M = M;
  c.L = L;
  c.pkind = p == 1.0 ? kSchatten1 : (p == 2.0 ? kSchatten2 : (std::isinf(p) ? kSchattenInf : kSchattenP));
  for (int j = 0; j < L; ++j) c.w[j] = weights[j];
  c.p = p;
  c.iters = iters;
  c.logits = logits;
  c.every = every;
  c.tol = tol;
  c.warm = warm;
  c.graph = graph;
  c.g4s = g4s;
  return SEGSALSA_OK;
}

segsalsa_status validate_image(int K, int H, int W, double lambda, double mu) {
  if (K < 2) return fail(SEGSALSA_ERR_INVALID_ARG, "K = %d must be >= 2", K);
  if (K > kMaxK) return fail(SEGSALSA_ERR_UNSUPPORTED, "K = %d exceeds %d", K, kMaxK);
  if (H < 1 || W < 1) return fail(SEGSALSA_ERR_INVALID_ARG, "H = %d, W = %d must be >= 1", H, W);
  if ((long long)H * W < 2) return fail(SEGSALSA_ERR_INVALID_ARG, "image must have >= 2 pixels");
  if (H > kMaxSide || W > kMaxSide) return fail(SEGSALSA_ERR_UNSUPPORTED, "H = %d, W = %d exceed %d", H, W, kMaxSide);
  if (!std::isfinite(lambda) || lambda < 0.0) return fail(SEGSALSA_ERR_INVALID_ARG, "lambda = %g", lambda);
  if (!std::isfinite(mu) || !(mu > 0.0)) return fail(SEGSALSA_ERR_INVALID_ARG, "mu = %g", mu);
  return SEGSALSA_OK;
}

segsalsa_status validate_problem(const segsalsa_problem* pr, segsalsa_precision prec, Common& c) {
  if (!pr) return fail(SEGSALSA_ERR_INVALID_ARG, "problem is NULL");
  segsalsa_status s = validate_image(pr->K, pr->H, pr->W, pr->lambda, pr->mu);
  if (s != SEGSALSA_OK) return s;
  return validate_common(pr->patch_radius, pr->patch_weights, pr->schatten_p, pr->iters, pr->input_is_logits,
                         pr->residual_every, pr->tol, pr->warm_start, pr->use_graph, pr->g4_simplex, prec, c);
}

// ---------------------------------------------------------------------------
// Per-image plan: tile grid, FFT factorisations and launch shapes, and the
// layout of the image's region of the workspace (offsets from its base).
// ---------------------------------------------------------------------------
// batch: the image is one of several solved together; the FFT blocking that
// the tuning entry leaves open then depends only on the transform length
// (rows or columns per workgroup, threads and elements per thread), not on
// how many workgroups the image alone would fill, so that the images of
// one length share a launch.
segsalsa_status plan_with(int K, int H, int W, const Common& c, const segsalsa_tuning& tn, Plan& p,
                          bool batch = false) {
  p.fp64 = c.fp64;
  p.ts = c.ts;
  p.K = K; p.H = H; p.W = W; p.M = c.M;
  p.L = c.L;
  p.P = (K + 1) / 2;
  p.g4s = c.g4s;
  p.tuned = false;
  // prox workgroup: the tuned classes per wavefront, else the fewest whose
  // register budget allows ceil(K/kpw) wavefronts
  p.kpw = 0;
  p.pf = tn.prefetch != 0;
  if (p.pf && (tn.classes_per_wave != 2 || !prox_has_prefetch_rt(p.fp64, p.M, 2)))
    return fail(SEGSALSA_ERR_UNSUPPORTED, "the prefetching prox kernel is built for FP32, 2 classes per wavefront, "
                "patch radius <= 2");
  for (int kpw : {1, 2, 4}) {
    if (tn.classes_per_wave > 0 && kpw != tn.classes_per_wave) continue;
    const int nw = ceil_div(K, kpw);
    if (nw <= 16 && nw * 64 <= prox_max_threads_rt(p.fp64, p.M, kpw, p.pf)) {
      p.kpw = kpw;
      p.nw = nw;
      break;
    }
  }
  if (p.kpw == 0) {
    if (tn.classes_per_wave > 0)
      return fail(SEGSALSA_ERR_UNSUPPORTED, "K = %d, M = %d: %d classes per wavefront do not fit one workgroup", K,
                  p.M, tn.classes_per_wave);
    p.kpw = 4;
    p.nw = ceil_div(K, 4);
    if (p.nw * 64 > prox_max_threads_rt(p.fp64, p.M, 4))
      return fail(SEGSALSA_ERR_UNSUPPORTED, "K = %d, M = %d do not fit one workgroup", K, p.M);
  }
  p.anw = p.akpw = 0;
  p.adj_lds = 0;
  if (c.grad) {
    for (int kpw : {1, 2, 4}) {
      const int nw = ceil_div(K, kpw);
      if (nw <= 16 && nw * 64 <= adj_max_threads_rt(p.fp64, p.M, kpw)) {
        p.akpw = kpw;
        p.anw = nw;
        break;
      }
    }
    if (p.akpw == 0) {
      p.akpw = 4;
      p.anw = ceil_div(K, 4);
      if (p.anw * 64 > adj_max_threads_rt(p.fp64, p.M, 4))
        return fail(SEGSALSA_ERR_UNSUPPORTED, "K = %d, M = %d do not fit one adjoint workgroup", K, p.M);
    }
  }
  if (!choose_tiles(p, tn.tile_rows, tn.tile_cols)) {
    if (tn.tile_rows > 0)
      return fail(SEGSALSA_ERR_UNSUPPORTED, "tile %dx%d does not fit LDS or the fold lists for K = %d, M = %d",
                  tn.tile_rows, tn.tile_cols, K, p.M);
    return fail(SEGSALSA_ERR_UNSUPPORTED, "no tile shape fits LDS for K = %d, M = %d", K, p.M);
  }
  const size_t cs = 2 * p.ts;
  p.frow = make_fft_plan(W);
  p.fcol = make_fft_plan(H);
  // Bluestein lengths of 64 .. 4096 run their convolution FFTs on the
  // fixed-structure engine (unless the general kernels are asked for)
  p.row_blu = p.frow.blu && p2_length(p.frow.M) && !tn.generic_fft;
  p.col_blu = p.fcol.blu && p2_length(p.fcol.M) && !tn.generic_fft;
  // the general kernels' Bluestein needs scratch next to the data; where
  // that exceeds LDS, keep the direct stages
  if (!p.row_blu && p.frow.blu && ((size_t)W + p.frow.M) * cs > kLdsBudget) p.frow.blu = 0;
  if (!p.col_blu && p.fcol.blu && ((size_t)H + p.fcol.M) * cs > kLdsBudget) p.fcol.blu = 0;
  // FFT workgroups.  Rows: whole rows plus the twiddle table (or the
  // Bluestein scratch) in LDS, about 2048 (FP32) / 1024 (FP64) elements per
  // workgroup at about 8 per thread (a radix-8 stage then keeps every thread
  // busy), but no fewer than two workgroups per compute unit when the image
  // has the rows.  Columns: blocks of adjacent columns so that each row of
  // a block is one contiguous run, at most 80 KB of LDS (two workgroups per
  // compute unit) and at least one workgroup per compute unit.
  // Power-of-two lengths 64 .. 4096 (without Bluestein) take the kernels
  // whose transform structure is fixed at compile time: N / 16 threads per
  // transform, about 256 threads per row workgroup and 512 per column
  // workgroup (FP64: 256), each transform in its own padded LDS region.
  // Bluestein lengths take the same engine over their convolution length M.
  const int maxthr_p2 = p.fp64 ? kFftNarrowThreads : kFftMaxThreads;
  p.row_p2 = p.row_blu ? p.frow.M : (!p.frow.blu && p2_length(W) && !tn.generic_fft ? W : 0);
  p.col_p2 = p.col_blu ? p.fcol.M : (!p.fcol.blu && p2_length(H) && !tn.generic_fft ? H : 0);
  if (p.row_p2) {
    const int tpt = p.row_p2 / 16;
    // default: about 256 threads, at least one wavefront, and two workgroups per CU when the image has the rows
    long long rpb = tn.rows_per_block > 0 ? std::min<long long>(tn.rows_per_block, H)
                    : batch             ? std::max(1, 256 / tpt)
                                        : std::min<long long>(H, std::max<long long>(std::max(1, 64 / tpt),
                                                                                    std::min<long long>(256 / tpt,
                                                                                                        (long long)p.P * H /
                                                                                                            (2 * kTargetGroups))));
    const long long thr = rpb * tpt;
    const size_t lds = (size_t)rpb * p2_region(p.row_p2) * cs;
    if (thr > maxthr_p2 || lds > kLdsBudget || (tn.row_threads > 0 && tn.row_threads != thr))
      return fail(SEGSALSA_ERR_UNSUPPORTED, "%lld rows of %d per workgroup (%lld threads, %zu bytes of LDS) do not fit",
                  rpb, W, thr, lds);
    p.rows_per_block = (int)rpb;
    p.row_threads = (int)thr;
    p.row_ept = 0;
    p.row_lds = lds;
  } else {
    const int Lr = p.frow.blu ? p.frow.M : W;      // elements per row inside the transform
    auto lds_of = [&](long long rpb) {
      return ((size_t)rpb * W + (p.frow.blu ? (size_t)rpb * Lr : (size_t)W)) * cs;
    };
    const long long nrows = (long long)p.P * H;
    long long rpb;
    const int rbudget = p.fp64 ? 1024 : 2048;   // elements per workgroup
    if (tn.rows_per_block > 0) {
      rpb = std::min<long long>(tn.rows_per_block, H);
    } else {
      rpb = std::max<long long>(1, rbudget / Lr);
      if (!batch) rpb = std::min<long long>(rpb, std::max<long long>(1, nrows / (2 * kTargetGroups)));
      rpb = std::max<long long>(1, std::min<long long>(rpb, H));
      while (rpb > 1 && (rpb * Lr > (long long)kFftEptMax * kFftMaxThreads || lds_of(rpb) > kLdsBudget)) --rpb;
    }
    if (rpb * Lr > (long long)kFftEptMax * kFftMaxThreads || lds_of(rpb) > kLdsBudget)
      return fail(SEGSALSA_ERR_UNSUPPORTED, "%lld rows of %d per FFT workgroup do not fit", rpb, W);
    const long long items = rpb * Lr;
    // in a batch, every row workgroup that holds the budget has the same shape
    const bool uniform = batch && tn.row_threads <= 0 && items <= rbudget;
    int thr = tn.row_threads > 0 ? tn.row_threads : uniform ? rbudget / 8 : fft_threads_for(items, 8);
    int ept = uniform ? 8 : fft_ept(items, thr);
    if (ept == 0) {
      if (tn.row_threads > 0)
        return fail(SEGSALSA_ERR_UNSUPPORTED, "%d row threads hold at most 16 of %lld elements each", thr, items);
      thr = fft_threads_for(items, kFftEptMax);
      ept = fft_ept(items, thr);
    }
    p.rows_per_block = (int)rpb;
    p.row_threads = thr;
    p.row_ept = ept;
    p.row_lds = lds_of(rpb);
  }
  // The recursions' FP32 rounding grows like eps / (1 - rho): at the largest
  // rho (kx = 0), 1 - rho falls below kTriMinGap once Wsum exceeds ~300, and
  // FP32 solves with such weights take the DFT column pass, whose error does
  // not depend on rho.
  double wsum = 0.0;
  for (int j = 0; j < c.L; ++j) {
    const double cj = c.fp64 ? c.w[j] : (double)(float)c.w[j];
    wsum += cj * cj;
  }
  const double a0 = 3.0 + 2.0 * wsum;
  const double rho0 = 2.0 * wsum / (a0 + std::sqrt(std::max(a0 * a0 - 4.0 * wsum * wsum, 0.0)));
  p.col_tri = !tn.col_dft && (c.fp64 || 1.0 - rho0 >= kTriMinGap);
  // a tuned column blocking is for the pass it names: kept for that pass only
  const bool col_tuned = p.col_tri || tn.col_dft;
  const int col_cpb = col_tuned ? tn.cols_per_block : 0, col_thr = col_tuned ? tn.col_threads : 0;
  if (p.col_tri) {
    // The tridiagonal recursions: lpt rows per thread, ceil(H / lpt) threads
    // per column; about 512 threads of adjacent columns per workgroup (fewer
    // for a single image too small to fill the GPU with them); in a batch,
    // 512 threads for every column length.
    const int lpt = p.fp64 ? 16 : 32;
    const int tpc = ceil_div(H, lpt);
    long long cb;
    if (col_cpb > 0) {
      cb = std::min<long long>(col_cpb, W);
    } else {
      cb = std::max(1, kTriThreads / tpc);
      if (!batch) {
        cb = std::min<long long>(cb, W);
        while (cb > 1 && (long long)p.P * ceil_div(W, (int)cb) < 2 * kTargetGroups) cb = (cb + 1) / 2;
      }
    }
    const long long need = cb * tpc;
    long long thr = col_thr > 0 ? col_thr
                    : batch && col_cpb <= 0 && need <= kTriThreads ? kTriThreads
                                                                             : (need + 63) / 64 * 64;
    if (thr < need || thr > kFftMaxThreads)
      return fail(SEGSALSA_ERR_UNSUPPORTED, "%lld columns of %d chunks need %lld threads (%lld given, at most %d)", cb,
                  tpc, need, thr, kFftMaxThreads);
    p.col_p2 = 0;
    p.col_blu = false;
    p.cols_per_block = (int)cb;
    p.col_threads = (int)thr;
    p.col_ept = lpt;
    p.col_lds = tri_lds((int)thr, p.ts);
  } else if (p.col_p2) {
    const int tpt = p.col_p2 / 16;
    // default: about 512 threads (FP64: 256), at least one wavefront, one workgroup per CU when there are the columns
    long long cb = col_cpb > 0 ? std::min<long long>(col_cpb, W)
                   : batch               ? std::max(1, (p.fp64 ? 256 : 512) / tpt)
                                         : std::min<long long>(W, std::max<long long>(std::max(1, 64 / tpt),
                                                                                     std::min<long long>((p.fp64 ? 256 : 512) / tpt,
                                                                                                         (long long)p.P * W /
                                                                                                             kTargetGroups)));
    const long long thr = cb * tpt;
    const size_t lds = (size_t)cb * p2_region(p.col_p2) * cs;
    const int maxthr_col = p.col_blu ? kFftNarrowThreads : maxthr_p2;   // the Bluestein column kernel's bound
    if (thr > maxthr_col || lds > kLdsBudget || (col_thr > 0 && col_thr != thr))
      return fail(SEGSALSA_ERR_UNSUPPORTED,
                  "%lld columns of %d per workgroup (%lld threads, %zu bytes of LDS) do not fit", cb, H, thr, lds);
    p.cols_per_block = (int)cb;
    p.col_threads = (int)thr;
    p.col_ept = 0;
    p.col_lds = lds;
  } else {
    const int Lc = p.fcol.blu ? p.fcol.M : H;
    auto lds_of = [&](long long cb) {
      return ((size_t)cb * H + (p.fcol.blu ? (size_t)cb * Lc : (size_t)H)) * cs;
    };
    long long cb;
    const int cbudget = 4096;   // elements per workgroup of a batch's uniform column shape
    if (col_cpb > 0) {
      cb = std::min<long long>(col_cpb, W);
    } else {
      cb = 1;
      const long long cmax = p.fp64 ? 8 : 16;   // 128-byte runs
      while (cb * 2 <= cmax && cb * 2 <= W && lds_of(cb * 2) <= 80 * 1024 &&
             cb * 2 * Lc <= (batch ? cbudget : (long long)kFftEptMax * kFftMaxThreads) &&
             (batch || (long long)p.P * ceil_div(W, (int)(cb * 2)) >= kTargetGroups))
        cb *= 2;
    }
    if (cb * Lc > (long long)kFftEptMax * kFftMaxThreads || lds_of(cb) > kLdsBudget)
      return fail(SEGSALSA_ERR_UNSUPPORTED, "%lld columns of %d per FFT workgroup do not fit", cb, H);
    const long long items = cb * Lc;
    // in a batch, every column workgroup within the budget has the same shape
    const bool uniform = batch && col_thr <= 0 && items <= cbudget;
    int thr = col_thr > 0 ? col_thr : uniform ? cbudget / 8 : fft_threads_for(items, 8);
    int ept = uniform ? 8 : fft_ept(items, thr);
    if (ept == 0) {
      if (col_thr > 0)
        return fail(SEGSALSA_ERR_UNSUPPORTED, "%d column threads hold at most 16 of %lld elements each", thr, items);
      thr = fft_threads_for(items, kFftEptMax);
      ept = fft_ept(items, thr);
    }
    p.cols_per_block = (int)cb;
    p.col_threads = thr;
    p.col_ept = ept;
    p.col_lds = lds_of(cb);
  }
  const size_t nt = (size_t)p.g.ntiles();
  size_t off = 0;
  p.off_flags = off; off = align_up(off + 64);
  p.off_twW = off; off = align_up(off + (size_t)W * cs);
  p.off_twH = off; off = align_up(off + (size_t)H * cs);
  p.off_sx = off; off = align_up(off + (size_t)W * 8);
  p.off_sy = off; off = align_up(off + (size_t)H * 8);
  p.off_frow = off; off = align_up(off + (size_t)H * kFoldStride * 4);
  p.off_fcol = off; off = align_up(off + (size_t)W * kFoldStride * 4);
  const size_t per_step = (size_t)K * 64 * p.ts;
  p.off_phat = off; off = align_up(off + nt * p.g.steps * per_step);
  p.off_dm = off; off = align_up(off + nt * p.g.steps * per_step * 3);
  p.off_d2 = off; off = align_up(off + nt * p.g.steps * per_step * 2 * p.L);
  off += kAccGuard;   // guard bands: the vector fold's masked loads reach a few elements beyond the partial sums
  p.off_acc = off; off = align_up(off + nt * (size_t)K * p.g.ER * p.g.EC * p.ts + kAccGuard);
  p.off_spec = off; off = align_up(off + (size_t)p.P * H * W * cs);
  p.off_zprev = off; off = align_up(off + (size_t)K * H * W * p.ts);
  p.off_restile = off; off = align_up(off + nt * 8);
  p.npartial = std::max<int>(kDiagBlocks, (int)(((size_t)H * W + 255) / 256));
  p.off_partial = off; off = align_up(off + (size_t)p.npartial * 8);
  p.off_out = off; off = align_up(off + 4 * 8);
  // Bluestein tables (only for lengths that use it)
  p.off_chW = off; off = align_up(off + (p.frow.blu ? (size_t)W * cs : 0));
  p.off_chH = off; off = align_up(off + (p.fcol.blu ? (size_t)H * cs : 0));
  p.off_bfW = off; off = align_up(off + (size_t)p.frow.M * cs);
  p.off_bfH = off; off = align_up(off + (size_t)p.fcol.M * cs);
  p.off_twMW = off; off = align_up(off + (size_t)p.frow.M * cs);
  p.off_twMH = off; off = align_up(off + (size_t)p.fcol.M * cs);
  p.total = off;
  return SEGSALSA_OK;
}

// Per-image plan: the tuned entry of the shape if there is one, the solve is
// of one image and the entry fits this problem (forward solves only: the
// differentiable solve sizes its tiles for the reverse sweep too, and the
// simplex g4 needs more LDS), else the planner's own choices.  The entries
// are measured with the image alone on the device; the images of a batch
// share it, and take the planner's batch shapes (FFT blocking by transform
// length only), which group into few, full launches.
void log_plan(const Plan& p) {
  const int K = p.K, H = p.H, W = p.W;
  if (const char* lg = std::getenv("SEGSALSA_LOG")) {
    if (lg[0] == '1')
      std::fprintf(stderr,
                   "[segsalsa] plan %s K=%d H=%d W=%d M=%d%s: tiles %dx%d (max %dx%d, %d tiles, %d steps), prox nw=%d "
                   "kpw=%d%s lds=%zu; rows/block=%d threads=%d ept=%d engine=%d%s lds=%zu; cols/block=%d "
                   "threads=%d ept=%d engine=%d%s lds=%zu; region %zu B\n",
                   p.fp64 ? "fp64" : "fp32", K, H, W, p.M, p.tuned ? " (tuned)" : "", p.g.ntr, p.g.ntc, p.g.TR,
                   p.g.TC, p.g.ntiles(), p.g.steps, p.nw, p.kpw, p.pf ? " prefetch" : "", p.prox_lds, p.rows_per_block,
                   p.row_threads, p.row_ept, p.row_p2, p.row_blu ? " bluestein" : "", p.row_lds, p.cols_per_block,
                   p.col_threads, p.col_ept, p.col_p2, p.col_blu ? " bluestein" : "", p.col_lds, p.total);
  }
}

segsalsa_status make_image_plan(int K, int H, int W, const Common& c, Plan& p, bool batch = false) {
  segsalsa_tuning tn{};
  if (!batch && !c.grad && tuning_lookup(K, H, W, c.M, c.fp64, tn)) {
    const std::string saved = g_last_error;
    if (plan_with(K, H, W, c, tn, p) == SEGSALSA_OK) {
      p.tuned = true;
      log_plan(p);
      return SEGSALSA_OK;
    }
    g_last_error = saved;
  }
  segsalsa_status s = plan_with(K, H, W, c, segsalsa_tuning{}, p, batch);
  if (s == SEGSALSA_OK) log_plan(p);
  return s;
}

template <typename T>
T* wsp(void* ws, size_t off) { return reinterpret_cast<T*>(reinterpret_cast<char*>(ws) + off); }

segsalsa_status check_ws(size_t need, const void* ws, size_t bytes) {
  if (!ws) return fail(SEGSALSA_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(SEGSALSA_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (bytes < need) return fail(SEGSALSA_ERR_WORKSPACE, "workspace %zu bytes < required %zu", bytes, need);
  return SEGSALSA_OK;
}

// ---------------------------------------------------------------------------
// Instrumentation: HIP events recorded on the caller's stream around each
// launch of a round, accumulated per phase when read back.
// ---------------------------------------------------------------------------
struct ProfState {
  std::mutex mu;
  bool on = false;
  std::vector<hipEvent_t> pool;
  struct Pending {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  double ms[SEGSALSA_NUM_PHASES] = {0};
  long long count[SEGSALSA_NUM_PHASES] = {0};
};
ProfState g_prof;

hipEvent_t prof_event_locked() {
  if (!g_prof.pool.empty()) {
    hipEvent_t e = g_prof.pool.back();
    g_prof.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Set while segsalsa_str_solve_noalloc runs on this thread: no event records
// (creating events may allocate).
thread_local bool g_no_alloc = false;

struct PhaseTimer {
  int phase;
  hipStream_t st;
  hipEvent_t a = nullptr;
  PhaseTimer(int ph, hipStream_t s) : phase(ph), st(s) {
    if (g_no_alloc) return;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    if (!g_prof.on) return;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return;
    a = prof_event_locked();
    if (a && hipEventRecord(a, st) != hipSuccess) a = nullptr;
  }
  void stop() {
    if (!a) return;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    hipEvent_t b = prof_event_locked();
    if (b && hipEventRecord(b, st) == hipSuccess) g_prof.pending.push_back({phase, a, b});
    a = nullptr;
  }
};


// ---------------------------------------------------------------------------
// Batch: image regions one after another, then the descriptor tables.
// ---------------------------------------------------------------------------
struct ImgRun {
  Plan plan;
  size_t base;        // offset of the image's workspace region
  double lambda, mu;
  size_t in_off, out_off;   // element offsets into the packed input / output
};

struct Batch {
  Common c{};
  std::vector<ImgRun> im;
  // prox, prox with residuals, row DFT, column solve, inverse row DFT, and for
  // the reverse sweep the row DFT of the cotangent and its inverse into rb
  size_t off_tab[7];
  size_t total;
};

template <typename T>
size_t desc_size(int which) {
  switch (which) {
    case 0:
    case 1: return sizeof(ProxArgs<T>);
    case 2: return sizeof(RowFwdArgs<T>);
    case 3: return sizeof(ColArgs<T>);
    case 5: return sizeof(RowFwdArgs<T>);
    default: return sizeof(RowInvArgs<T>);
  }
}

// force (autotuning, one image): plan with these shapes instead of the table's or the planner's.
segsalsa_status make_batch(int n, const int* K, const int* H, const int* W, const double* lam, const double* mu,
                           const Common& c, Batch& b, const segsalsa_tuning* force = nullptr) {
  b.c = c;
  b.im.resize(n);
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    segsalsa_status s = validate_image(K[i], H[i], W[i], lam[i], mu[i]);
    if (s != SEGSALSA_OK) return fail(s, "image %d: %s", i, segsalsa_last_error());
    s = force ? plan_with(K[i], H[i], W[i], c, *force, b.im[i].plan)
              : make_image_plan(K[i], H[i], W[i], c, b.im[i].plan, n > 1);
    if (s != SEGSALSA_OK) return s;
    b.im[i].base = off;
    b.im[i].lambda = lam[i];
    b.im[i].mu = mu[i];
    off = align_up(off + b.im[i].plan.total);
  }
  for (int t = 0; t < 7; ++t) {
    b.off_tab[t] = off;
    off = align_up(off + (size_t)n * (c.fp64 ? desc_size<double>(t) : desc_size<float>(t)));
  }
  b.total = off;
  return SEGSALSA_OK;
}

// Launch shapes for the active images: one launch per distinct workgroup
// shape of each kernel (the prox kernel by wavefronts and classes per
// wavefront, the FFT passes by threads and elements per thread), over the
// images of that shape, whose descriptors are contiguous in the tables.
struct LaunchSet {
  struct Group {
    int kpw, nw, first, count, blocks;
    size_t lds;
    bool pf;
  };
  struct FftGroup {
    int ept, threads, first, count, blocks;
    size_t lds;
    int p2;   // length of the fixed-structure engine, 0: general kernels
    bool blu;  // the engine runs Bluestein's convolution (p2 is its length)
    bool tri;  // columns: the tridiagonal recursions (ept rows per thread)
  };
  std::vector<Group> groups;
  std::vector<FftGroup> rgroups, cgroups;
  int nact = 0;
  bool nt = false;   // the prox launches stream the state past the caches
};

template <typename T>
FftTab<T> row_tab(const Plan& p, void* base) {
  FftTab<T> t;
  t.tw = wsp<C2<T>>(base, p.off_twW);
  t.chirp = wsp<C2<T>>(base, p.off_chW);
  t.bf = wsp<C2<T>>(base, p.off_bfW);
  t.twM = wsp<C2<T>>(base, p.off_twMW);
  return t;
}

template <typename T>
FftTab<T> col_tab(const Plan& p, void* base) {
  FftTab<T> t;
  t.tw = wsp<C2<T>>(base, p.off_twH);
  t.chirp = wsp<C2<T>>(base, p.off_chH);
  t.bf = wsp<C2<T>>(base, p.off_bfH);
  t.twM = wsp<C2<T>>(base, p.off_twMH);
  return t;
}

template <typename T>
hipError_t upload_tables(const Batch& b, void* ws, const std::vector<int>& active, void* const* zs,
                         const void* const* ins, LaunchSet& ls, hipStream_t st, void* const* adj_acc = nullptr,
                         void* const* adj_r = nullptr) {
  (void)ins;
  const Common& c = b.c;
  ls = LaunchSet();
  ls.nact = (int)active.size();
  // the per-pixel state a round streams through the prox kernel, all images
  size_t state = 0;
  for (int i : active) {
    const Plan& p = b.im[i].plan;
    state += (size_t)p.H * p.W * p.K * (4 * p.L + 9) * p.ts;
  }
  ls.nt = state > kStreamBytes;
  // prox: sort by (nw, kpw) so each group is one launch over a contiguous range
  std::vector<int> order(active);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    const Plan& px = b.im[x].plan;
    const Plan& py = b.im[y].plan;
    return px.nw != py.nw ? px.nw < py.nw : (px.kpw != py.kpw ? px.kpw < py.kpw : px.pf < py.pf);
  });
  std::vector<ProxArgs<T>> pa(order.size()), pb;
  for (size_t q = 0; q < order.size(); ++q) {
    const ImgRun& r = b.im[order[q]];
    const Plan& p = r.plan;
    void* base = wsp<char>(ws, r.base);
    if (ls.groups.empty() || ls.groups.back().nw != p.nw || ls.groups.back().kpw != p.kpw ||
        ls.groups.back().pf != p.pf)
      ls.groups.push_back({p.kpw, p.nw, (int)q, 0, 0, 0, p.pf});
    LaunchSet::Group& g = ls.groups.back();
    ProxArgs<T>& a = pa[q];
    std::memset(&a, 0, sizeof(a));
    a.block0 = g.blocks;
    a.g = p.g;
    a.K = p.K;
    a.nw = p.nw;
    a.z = reinterpret_cast<T*>(zs[order[q]]);
    a.phat = wsp<T>(base, p.off_phat);
    a.dm = wsp<T>(base, p.off_dm);
    a.d2 = wsp<T>(base, p.off_d2);
    a.dm_in = a.dm;
    a.d2_in = a.d2;
    a.acc = wsp<T>(base, p.off_acc);
    a.res_tile = nullptr;
    a.mu = r.mu;
    a.tau = r.lambda / r.mu;
    a.pkind = c.pkind;
    a.pval = c.p;
    a.g4s = c.g4s;
    for (int j = 0; j < c.L; ++j) a.c[j] = (T)c.w[j];
    g.count += 1;
    g.blocks += p.g.ntiles();
    g.lds = std::max(g.lds, p.prox_lds);
  }
  pb = pa;
  for (size_t q = 0; q < order.size(); ++q) {
    const ImgRun& r = b.im[order[q]];
    pb[q].res_tile = wsp<double>(wsp<char>(ws, r.base), r.plan.off_restile);
  }
  // FFT passes: the row tables (fold + row DFT, inverse row DFT) ordered by
  // the row workgroup shape, the column table by the column shape
  std::vector<int> rord(active), cord(active);
  std::stable_sort(rord.begin(), rord.end(), [&](int x, int y) {
    const Plan& px = b.im[x].plan;
    const Plan& py = b.im[y].plan;
    return std::tie(px.row_blu, px.row_p2, px.row_threads, px.row_ept) <
           std::tie(py.row_blu, py.row_p2, py.row_threads, py.row_ept);
  });
  std::stable_sort(cord.begin(), cord.end(), [&](int x, int y) {
    const Plan& px = b.im[x].plan;
    const Plan& py = b.im[y].plan;
    return std::tie(px.col_tri, px.col_blu, px.col_p2, px.col_threads, px.col_ept) <
           std::tie(py.col_tri, py.col_blu, py.col_p2, py.col_threads, py.col_ept);
  });
  std::vector<RowFwdArgs<T>> rf(active.size());
  std::vector<ColArgs<T>> ca(active.size());
  std::vector<RowInvArgs<T>> ri(active.size());
  double wsum = 0.0;
  for (int j = 0; j < c.L; ++j) {
    const double cj = (double)(T)c.w[j];  // the multiplier J applies, rounded to T
    wsum += cj * cj;
  }
  for (size_t q = 0; q < rord.size(); ++q) {
    const ImgRun& r = b.im[rord[q]];
    const Plan& p = r.plan;
    void* base = wsp<char>(ws, r.base);
    if (ls.rgroups.empty() || ls.rgroups.back().threads != p.row_threads || ls.rgroups.back().ept != p.row_ept ||
        ls.rgroups.back().p2 != p.row_p2 || ls.rgroups.back().blu != p.row_blu)
      ls.rgroups.push_back({p.row_ept, p.row_threads, (int)q, 0, 0, 0, p.row_p2, p.row_blu});
    LaunchSet::FftGroup& g = ls.rgroups.back();
    RowFwdArgs<T>& f = rf[q];
    std::memset(&f, 0, sizeof(f));
    f.block0 = g.blocks;
    f.g = p.g;
    f.K = p.K;
    f.P = p.P;
    f.rows_per_block = p.rows_per_block;
    f.vfold = vector_fold_fits(p.g, sizeof(T));
    f.acc = wsp<T>(base, p.off_acc);
    f.frow = wsp<int>(base, p.off_frow);
    f.fcol = wsp<int>(base, p.off_fcol);
    f.spec = wsp<C2<T>>(base, p.off_spec);
    f.tab = row_tab<T>(p, base);
    f.plan = p.frow;
    RowInvArgs<T>& v = ri[q];
    std::memset(&v, 0, sizeof(v));
    v.block0 = g.blocks;
    v.H = p.H; v.W = p.W; v.K = p.K; v.P = p.P;
    v.rows_per_block = p.rows_per_block;
    v.spec = f.spec;
    v.z = reinterpret_cast<T*>(zs[rord[q]]);
    v.tab = f.tab;
    v.plan = p.frow;
    g.count += 1;
    g.blocks += p.P * ceil_div(p.H, p.rows_per_block);
    g.lds = std::max(g.lds, p.row_lds);
  }
  for (size_t q = 0; q < cord.size(); ++q) {
    const ImgRun& r = b.im[cord[q]];
    const Plan& p = r.plan;
    void* base = wsp<char>(ws, r.base);
    if (ls.cgroups.empty() || ls.cgroups.back().threads != p.col_threads || ls.cgroups.back().ept != p.col_ept ||
        ls.cgroups.back().p2 != p.col_p2 || ls.cgroups.back().blu != p.col_blu || ls.cgroups.back().tri != p.col_tri)
      ls.cgroups.push_back({p.col_ept, p.col_threads, (int)q, 0, 0, 0, p.col_p2, p.col_blu, p.col_tri});
    LaunchSet::FftGroup& g = ls.cgroups.back();
    ColArgs<T>& k = ca[q];
    std::memset(&k, 0, sizeof(k));
    k.block0 = g.blocks;
    k.H = p.H; k.W = p.W; k.P = p.P;
    k.cols_per_block = p.cols_per_block;
    k.spec = wsp<C2<T>>(base, p.off_spec);
    k.tab = col_tab<T>(p, base);
    k.sx = wsp<double>(base, p.off_sx);
    k.sy = wsp<double>(base, p.off_sy);
    k.wsum = wsum;
    k.scale = 1.0 / ((double)p.H * (double)p.W);
    k.plan = p.fcol;
    g.count += 1;
    g.blocks += p.P * ceil_div(p.W, p.cols_per_block);
    g.lds = std::max(g.lds, p.col_lds);
  }
  hipError_t e;
  if (!pa.empty()) {
    if ((e = launch_store(wsp<char>(ws, b.off_tab[0]), pa.data(), pa.size() * sizeof(pa[0]), st)) != hipSuccess) return e;
    if ((e = launch_store(wsp<char>(ws, b.off_tab[1]), pb.data(), pb.size() * sizeof(pb[0]), st)) != hipSuccess) return e;
    if ((e = launch_store(wsp<char>(ws, b.off_tab[2]), rf.data(), rf.size() * sizeof(rf[0]), st)) != hipSuccess) return e;
    if ((e = launch_store(wsp<char>(ws, b.off_tab[3]), ca.data(), ca.size() * sizeof(ca[0]), st)) != hipSuccess) return e;
    if ((e = launch_store(wsp<char>(ws, b.off_tab[4]), ri.data(), ri.size() * sizeof(ri[0]), st)) != hipSuccess) return e;
    if (adj_acc && adj_r) {  // reverse sweep: fold the cotangent's partial sums, solve into rb
      for (size_t q = 0; q < rord.size(); ++q) {
        rf[q].acc = reinterpret_cast<const T*>(adj_acc[rord[q]]);
        ri[q].z = reinterpret_cast<T*>(adj_r[rord[q]]);
      }
      if ((e = launch_store(wsp<char>(ws, b.off_tab[5]), rf.data(), rf.size() * sizeof(rf[0]), st)) != hipSuccess)
        return e;
      if ((e = launch_store(wsp<char>(ws, b.off_tab[6]), ri.data(), ri.size() * sizeof(ri[0]), st)) != hipSuccess)
        return e;
    }
  }
  return hipSuccess;
}

// The z-update solve A z = rhs (eq. (12)) by the three FFT passes, with the
// row tables `fwd_tab` (fold + row DFT) and `inv_tab` (inverse row DFT).
// ev (autotuning): if given, ev[0] is recorded after the row DFT pass, ev[1]
// after the column pass and ev[2] after the inverse row pass.
template <typename T>
hipError_t enqueue_fft(const Batch& b, const LaunchSet& ls, void* ws, hipStream_t st, int fwd_tab, int inv_tab,
                       hipEvent_t* ev = nullptr) {
  hipError_t e = hipSuccess;
  // FP64 workgroups of at most 512 threads run the build with 256 VGPRs
  auto narrow = [](int threads) { return sizeof(T) == 8 && threads <= kFftNarrowThreads; };
  {
    PhaseTimer t1(1, st);
    const RowFwdArgs<T>* tab = wsp<RowFwdArgs<T>>(ws, b.off_tab[fwd_tab]);
    for (const auto& g : ls.rgroups)
      if ((e = g.blu  ? launch_rows_fwd_blu(tab + g.first, g.count, g.blocks, g.p2, g.threads, g.lds, st)
               : g.p2 ? launch_rows_fwd_p2(tab + g.first, g.count, g.blocks, g.p2, g.threads, g.lds, st)
                      : launch_rows_fwd(tab + g.first, g.count, g.blocks, g.ept, g.threads, narrow(g.threads), g.lds,
                                        st)) != hipSuccess)
        return e;
    t1.stop();
    if (ev && (e = hipEventRecord(ev[0], st)) != hipSuccess) return e;
  }
  {
    PhaseTimer t2(2, st);
    const ColArgs<T>* tab = wsp<ColArgs<T>>(ws, b.off_tab[3]);
    for (const auto& g : ls.cgroups)
      if ((e = g.tri  ? launch_cols_tri(tab + g.first, g.count, g.blocks, g.ept, g.threads, g.lds, st)
               : g.blu  ? launch_cols_blu(tab + g.first, g.count, g.blocks, g.p2, g.threads, g.lds, st)
               : g.p2 ? launch_cols_p2(tab + g.first, g.count, g.blocks, g.p2, g.threads, g.lds, st)
                      : launch_cols(tab + g.first, g.count, g.blocks, g.ept, g.threads, narrow(g.threads), g.lds, st)) !=
          hipSuccess)
        return e;
    t2.stop();
    if (ev && (e = hipEventRecord(ev[1], st)) != hipSuccess) return e;
  }
  {
    PhaseTimer t3(3, st);
    const RowInvArgs<T>* tab = wsp<RowInvArgs<T>>(ws, b.off_tab[inv_tab]);
    for (const auto& g : ls.rgroups)
      if ((e = g.blu  ? launch_rows_inv_blu(tab + g.first, g.count, g.blocks, g.p2, g.threads, g.lds, st)
               : g.p2 ? launch_rows_inv_p2(tab + g.first, g.count, g.blocks, g.p2, g.threads, g.lds, st)
                      : launch_rows_inv(tab + g.first, g.count, g.blocks, g.ept, g.threads, narrow(g.threads), g.lds,
                                        st)) != hipSuccess)
        return e;
    t3.stop();
    if (ev && (e = hipEventRecord(ev[2], st)) != hipSuccess) return e;
  }
  return e;
}

// ev (autotuning): if given, five events recorded before the prox launches,
// after them, and after each FFT pass.
template <typename T>
hipError_t enqueue_round(const Batch& b, const LaunchSet& ls, void* ws, hipStream_t st, bool residuals,
                         hipEvent_t* ev = nullptr) {
  if (ls.nact == 0) return hipSuccess;
  hipError_t e;
  if (ev && (e = hipEventRecord(ev[0], st)) != hipSuccess) return e;
  const ProxArgs<T>* ptab = wsp<ProxArgs<T>>(ws, b.off_tab[residuals ? 1 : 0]);
  {
    PhaseTimer t0(0, st);
    for (const auto& g : ls.groups) {
      // checked rounds (residuals) and the variants run the instantiation that has them,
      // which is built without the prefetch
      const bool var = b.c.pkind == kSchattenP || b.c.g4s || residuals;
      e = launch_prox(ptab + g.first, g.count, g.blocks, g.nw * 64, b.c.M, g.kpw, g.pf && !var, ls.nt, g.lds, var,
                      st);
      if (e != hipSuccess) return e;
    }
    t0.stop();
  }
  if (ev && (e = hipEventRecord(ev[1], st)) != hipSuccess) return e;
  return enqueue_fft<T>(b, ls, ws, st, 2, 4, ev ? ev + 2 : nullptr);
}

template <typename T>
DiagArgs<T> diag_args(const Batch& b, int i, void* ws, void* z) {
  const ImgRun& r = b.im[i];
  const Plan& p = r.plan;
  void* base = wsp<char>(ws, r.base);
  DiagArgs<T> da;
  std::memset(&da, 0, sizeof(da));
  da.g = p.g;
  da.K = p.K;
  da.pkind = b.c.pkind;
  da.pval = b.c.p;
  da.lambda = r.lambda;
  for (int j = 0; j < p.L; ++j) {
    da.cw[j] = (double)(T)b.c.w[j];
    da.wsum += da.cw[j] * da.cw[j];
  }
  da.z = reinterpret_cast<T*>(z);
  da.zprev = wsp<T>(base, p.off_zprev);
  da.phat = wsp<T>(base, p.off_phat);
  da.partial = wsp<double>(base, p.off_partial);
  da.out = wsp<double>(base, p.off_out);
  return da;
}

// Set-up (tables) of every image, initialisation unless `init` is false, and
// the upload of the launch descriptors.
template <typename T>
hipError_t enqueue_prepare(const Batch& b, void* ws, void* const* zs, const void* const* ins, hipStream_t st,
                           LaunchSet& ls, bool init, void* const* adj_acc = nullptr, void* const* adj_r = nullptr) {
  hipError_t e;
  const Common& c = b.c;
  const int n = (int)b.im.size();
  for (int i = 0; i < n; ++i) {
    const ImgRun& r = b.im[i];
    const Plan& p = r.plan;
    void* base = wsp<char>(ws, r.base);
    SetupArgs<T> sa;
    sa.g = p.g;
    sa.frow = wsp<int>(base, p.off_frow);
    sa.fcol = wsp<int>(base, p.off_fcol);
    sa.H = p.H;
    sa.W = p.W;
    sa.twW = wsp<C2<T>>(base, p.off_twW);
    sa.twH = wsp<C2<T>>(base, p.off_twH);
    sa.sx = wsp<double>(base, p.off_sx);
    sa.sy = wsp<double>(base, p.off_sy);
    sa.MW = p.frow.blu ? p.frow.M : 0;
    sa.MH = p.fcol.blu ? p.fcol.M : 0;
    sa.chW = wsp<C2<T>>(base, p.off_chW);
    sa.chH = wsp<C2<T>>(base, p.off_chH);
    sa.twMW = wsp<C2<T>>(base, p.off_twMW);
    sa.twMH = wsp<C2<T>>(base, p.off_twMH);
    if ((e = launch_setup(sa, st)) != hipSuccess) return e;
    if (p.frow.blu) {
      const FftTab<T> t = row_tab<T>(p, base);
      if ((e = launch_bluestein_table(p.frow, t, wsp<C2<T>>(base, p.off_bfW), st)) != hipSuccess) return e;
    }
    if (p.fcol.blu) {
      const FftTab<T> t = col_tab<T>(p, base);
      if ((e = launch_bluestein_table(p.fcol, t, wsp<C2<T>>(base, p.off_bfH), st)) != hipSuccess) return e;
    }
    if (init) {
      if ((e = launch_fill_zero(wsp<char>(base, p.off_flags), 64, st)) != hipSuccess) return e;
      if ((e = launch_fill_zero(wsp<char>(base, p.off_d2), p.off_acc - p.off_d2, st)) != hipSuccess) return e;
      InitArgs<T> ia;
      ia.g = p.g;
      ia.K = p.K;
      ia.is_logits = c.logits;
      ia.input = reinterpret_cast<const T*>(ins[i]);
      ia.z = reinterpret_cast<T*>(zs[i]);
      ia.phat = wsp<T>(base, p.off_phat);
      ia.dm = wsp<T>(base, p.off_dm);
      ia.flags = wsp<int>(base, p.off_flags);
      if ((e = launch_init(ia, st)) != hipSuccess) return e;
    }
  }
  std::vector<int> active(n);
  for (int i = 0; i < n; ++i) active[i] = i;
  return upload_tables<T>(b, ws, active, zs, ins, ls, st, adj_acc, adj_r);
}

// Set-up and initialisation of every image, then all rounds.
template <typename T>
hipError_t enqueue_solve(const Batch& b, void* ws, void* const* zs, const void* const* ins, hipStream_t st,
                         LaunchSet& ls) {
  hipError_t e;
  const Common& c = b.c;
  if ((e = enqueue_prepare<T>(b, ws, zs, ins, st, ls, !c.warm)) != hipSuccess) return e;
  if (c.every == 0) {
    for (int it = 0; it < c.iters; ++it)
      if ((e = enqueue_round<T>(b, ls, ws, st, false)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Rounds with residual checks: every `every` rounds (and after the last) the
// residuals of each active image are read back; with tol > 0, images whose
// primal and dual residuals are both <= tol stop (the stopping rule of Sec. 4)
// and the launch tables are rebuilt without them.
template <typename T>
segsalsa_status run_checked(const Batch& b, void* ws, void* const* zs, const void* const* ins, hipStream_t st,
                            LaunchSet& ls, segsalsa_stats* stats) {
  const Common& c = b.c;
  const int n = (int)b.im.size();
  hipError_t e;
  std::vector<int> active(n), done(n, 0);
  std::vector<double> rp(n, 0.0), rd(n, 0.0);
  for (int i = 0; i < n; ++i) active[i] = i;
  std::vector<double> host(2 * (size_t)n);
  for (int it = 0; it < c.iters && !active.empty(); ++it) {
    const bool checked = (it + 1) % c.every == 0 || it + 1 == c.iters;
    if (checked)
      for (const int i : active) {
        const Plan& p = b.im[i].plan;
        DiagArgs<T> da = diag_args<T>(b, i, ws, zs[i]);
        if ((e = launch_copy(da.z, da.zprev, (size_t)p.K * p.H * p.W, st)) != hipSuccess) return hip_fail(e, "copy z");
      }
    if ((e = enqueue_round<T>(b, ls, ws, st, checked)) != hipSuccess) return hip_fail(e, "round");
    for (const int i : active) done[i] = it + 1;
    if (!checked) continue;
    for (size_t q = 0; q < active.size(); ++q) {
      const int i = active[q];
      const Plan& p = b.im[i].plan;
      DiagArgs<T> da = diag_args<T>(b, i, ws, zs[i]);
      void* base = wsp<char>(ws, b.im[i].base);
      if ((e = launch_reduce(wsp<double>(base, p.off_restile), p.g.ntiles(), da.out, 0, st)) != hipSuccess)
        return hip_fail(e, "residual reduce");
      if ((e = launch_dual_res(da, st)) != hipSuccess) return hip_fail(e, "dual residual");
      if ((e = hipMemcpyAsync(&host[2 * q], da.out, 2 * sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess)
        return hip_fail(e, "residual copy");
    }
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "stream sync");
    std::vector<int> still;
    for (size_t q = 0; q < active.size(); ++q) {
      const int i = active[q];
      rp[i] = std::sqrt(std::max(host[2 * q], 0.0));
      rd[i] = b.im[i].mu * std::sqrt(std::max(host[2 * q + 1], 0.0));
      if (!(c.tol > 0.0 && rp[i] <= c.tol && rd[i] <= c.tol)) still.push_back(i);
    }
    if (still.size() != active.size()) {
      active.swap(still);
      if ((e = upload_tables<T>(b, ws, active, zs, ins, ls, st)) != hipSuccess) return hip_fail(e, "tables");
    }
  }
  for (int i = 0; i < n; ++i) {
    stats[i].primal_res = rp[i];
    stats[i].dual_res = rd[i];
    stats[i].rounds_done = done[i];
  }
  return SEGSALSA_OK;
}

// Fill stats after the rounds: input flags, and the objective when residuals were asked for.
template <typename T>
segsalsa_status finish_stats(const Batch& b, void* ws, void* const* zs, hipStream_t st, segsalsa_stats* stats) {
  const int n = (int)b.im.size();
  hipError_t e;
  std::vector<int> flags(n, 0);
  std::vector<double> obj(n, 0.0);
  for (int i = 0; i < n; ++i) {
    const ImgRun& r = b.im[i];
    void* base = wsp<char>(ws, r.base);
    if (b.c.every > 0) {
      DiagArgs<T> da = diag_args<T>(b, i, ws, zs[i]);
      if ((e = launch_objective(da, st)) != hipSuccess) return hip_fail(e, "objective");
      if ((e = hipMemcpyAsync(&obj[i], da.out + 2, sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess)
        return hip_fail(e, "objective copy");
    }
    if ((e = hipMemcpyAsync(&flags[i], wsp<int>(base, r.plan.off_flags), sizeof(int), hipMemcpyDeviceToHost, st)) !=
        hipSuccess)
      return hip_fail(e, "flags copy");
  }
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "stream sync");
  for (int i = 0; i < n; ++i) {
    stats[i].flags = flags[i];
    stats[i].objective = obj[i];
  }
  return SEGSALSA_OK;
}

// ---------------------------------------------------------------------------
// Whole-solve hipGraphs: captured once per (workspace, buffers, problem) and
// replayed, so a solve is one graph launch.
// ---------------------------------------------------------------------------
struct GraphEntry {
  std::vector<unsigned char> key;
  int device;
  hipGraphExec_t exec;
};
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;   // most recent last
constexpr size_t kGraphCache = 8;

void key_add(std::vector<unsigned char>& k, const void* p, size_t n) {
  const unsigned char* c = reinterpret_cast<const unsigned char*>(p);
  k.insert(k.end(), c, c + n);
}

std::vector<unsigned char> graph_key(const Batch& b, void* ws, void* const* zs, const void* const* ins) {
  std::vector<unsigned char> k;
  const Common& c = b.c;   // named fields only (no padding bytes, only the L multipliers in use)
  const int ci[] = {c.fp64 ? 1 : 0, c.M, c.L, c.pkind, c.iters, c.logits, c.every, c.warm, c.graph, c.g4s};
  key_add(k, ci, sizeof(ci));
  key_add(k, c.w, sizeof(double) * (size_t)c.L);
  key_add(k, &c.p, sizeof(c.p));
  key_add(k, &c.tol, sizeof(c.tol));
  key_add(k, &ws, sizeof(ws));
  for (size_t i = 0; i < b.im.size(); ++i) {
    const ImgRun& r = b.im[i];
    key_add(k, &r.plan.K, sizeof(int));
    key_add(k, &r.plan.H, sizeof(int));
    key_add(k, &r.plan.W, sizeof(int));
    key_add(k, &r.lambda, sizeof(double));
    key_add(k, &r.mu, sizeof(double));
    key_add(k, &zs[i], sizeof(void*));
    key_add(k, &ins[i], sizeof(void*));
  }
  // plan choices that the tuning table can change
  for (size_t i = 0; i < b.im.size(); ++i) {
    const Plan& p = b.im[i].plan;
    const int pi[] = {p.g.ntr,          p.g.ntc,       p.kpw,            p.pf ? 1 : 0, p.row_p2,
                      p.rows_per_block, p.row_threads, p.cols_per_block, p.col_threads, p.col_p2,
                      p.row_blu ? 1 : 0, p.col_blu ? 1 : 0, p.col_tri ? 1 : 0};
    key_add(k, pi, sizeof(pi));
  }
  return k;
}

hipStream_t capture_stream(int device) {
  static std::mutex mu;
  static std::vector<hipStream_t> streams;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)streams.size() <= device) streams.resize(device + 1, nullptr);
  if (!streams[device]) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    streams[device] = s;
  }
  return streams[device];
}

template <typename T>
segsalsa_status run_graph(const Batch& b, void* ws, void* const* zs, const void* const* ins, hipStream_t st) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::vector<unsigned char> key = graph_key(b, ws, zs, ins);
  std::lock_guard<std::mutex> lk(g_graph_mu);
  for (size_t i = 0; i < g_graphs.size(); ++i) {
    if (g_graphs[i].device == dev && g_graphs[i].key == key) {
      GraphEntry ent = g_graphs[i];
      g_graphs.erase(g_graphs.begin() + i);
      g_graphs.push_back(ent);
      e = hipGraphLaunch(ent.exec, st);
      return e == hipSuccess ? SEGSALSA_OK : hip_fail(e, "hipGraphLaunch");
    }
  }
  hipStream_t cs = capture_stream(dev);
  if (!cs) return fail(SEGSALSA_ERR_DEVICE, "cannot create the capture stream");
  LaunchSet ls;
  if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed)) != hipSuccess) return hip_fail(e, "begin capture");
  hipError_t ee = enqueue_solve<T>(b, ws, zs, ins, cs, ls);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cs, &graph);
  if (ee != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_fail(ee, "capture");
  }
  if (e != hipSuccess) return hip_fail(e, "end capture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(e, "graph instantiate");
  if (g_graphs.size() >= kGraphCache) {
    (void)hipGraphExecDestroy(g_graphs.front().exec);
    g_graphs.erase(g_graphs.begin());
  }
  g_graphs.push_back({key, dev, exec});
  e = hipGraphLaunch(exec, st);
  return e == hipSuccess ? SEGSALSA_OK : hip_fail(e, "hipGraphLaunch");
}

template <typename T>
segsalsa_status solve_batch_t(const Batch& b, void* ws, void* const* zs, const void* const* ins, hipStream_t st,
                              segsalsa_stats* stats) {
  const int n = (int)b.im.size();
  if (b.c.graph) {
    segsalsa_status s = run_graph<T>(b, ws, zs, ins, st);
    if (s != SEGSALSA_OK) return s;
  } else {
    LaunchSet ls;
    hipError_t e = enqueue_solve<T>(b, ws, zs, ins, st, ls);
    if (e != hipSuccess) return hip_fail(e, "enqueue");
    if (b.c.every > 0) {
      segsalsa_status s = run_checked<T>(b, ws, zs, ins, st, ls, stats);
      if (s != SEGSALSA_OK) return s;
    }
  }
  if (stats) {
    if (b.c.every == 0)
      for (int i = 0; i < n; ++i) {
        std::memset(&stats[i], 0, sizeof(stats[i]));
        stats[i].rounds_done = b.c.iters;
      }
    return finish_stats<T>(b, ws, zs, st, stats);
  }
  return SEGSALSA_OK;
}

segsalsa_status single_batch(const segsalsa_problem* pr, segsalsa_precision prec, Batch& b) {
  Common c{};
  segsalsa_status s = validate_problem(pr, prec, c);
  if (s != SEGSALSA_OK) return s;
  return make_batch(1, &pr->K, &pr->H, &pr->W, &pr->lambda, &pr->mu, c, b);
}

template <typename T>
hipError_t run_state(const Plan& p, void* ws, int to_canon, const void* ph, const void* d1, const void* d2,
                     const void* d3, const void* d4, hipStream_t st) {
  StateArgs<T> a;
  a.g = p.g;
  a.K = p.K;
  a.L = p.L;
  a.to_canonical = to_canon;
  a.phat_t = wsp<T>(ws, p.off_phat);
  a.dm_t = wsp<T>(ws, p.off_dm);
  a.d2_t = wsp<T>(ws, p.off_d2);
  a.phat = const_cast<T*>(reinterpret_cast<const T*>(ph));
  a.d1 = const_cast<T*>(reinterpret_cast<const T*>(d1));
  a.d2 = const_cast<T*>(reinterpret_cast<const T*>(d2));
  a.d3 = const_cast<T*>(reinterpret_cast<const T*>(d3));
  a.d4 = const_cast<T*>(reinterpret_cast<const T*>(d4));
  return launch_state(a, st);
}

// ---------------------------------------------------------------------------
// Differentiable solve: forward rounds with checkpoints, then the reverse
// sweep.  Workspace = the single-image solve region and its tables, then
//   zw      [K][H][W]  z of the rounds being run
//   r       [K][H][W]  rb = A^{-1} zb' of the reverse round
//   bst     cotangents of the multipliers (the layout of dm, d2)
//   pbar    tile layout, cotangent of p_hat from the data term
//   bacc    grown-tile partial sums of the cotangent of z
//   gpart   [tiles][L + 2] FP64 per-tile parameter totals, gtot [L + 2]
//   ck      ceil(iters / S) checkpoints (z, multipliers) at rounds 0, S, 2S, ...
//   zN      z after the last round
//   seg     S - 1 slots of (z, multipliers) recomputed inside one segment
// ---------------------------------------------------------------------------
struct GradLayout {
  Batch b;
  int S = 1, nck = 1, nseg = 0;
  size_t zbytes = 0, sbytes = 0;
  size_t off_zw, off_r, off_bst, off_pbar, off_bacc, off_gpart, off_gtot, off_ck, off_zN, off_seg, total;
  size_t ck(int i) const { return off_ck + (size_t)i * (zbytes + sbytes); }
  size_t seg(int i) const { return off_seg + (size_t)i * (zbytes + sbytes); }
};

// checkpoint_every = 0: the smallest interval whose kept states, ceil(N / S)
// checkpoints and S - 1 recomputed ones, fit in kAutoStateBytes (S = 1 keeps
// every state and recomputes nothing), else ceil(sqrt(N)).
constexpr size_t kAutoStateBytes = (size_t)8 << 30;

int auto_interval(int N, size_t state_bytes) {
  if (N <= 1) return 1;
  for (int S = 1; S <= N; ++S) {
    const size_t kept = (size_t)ceil_div(N, S) + (size_t)(S - 1);
    if (kept * state_bytes <= kAutoStateBytes) return S;
    if ((long long)S * S >= N) break;   // past the minimum of ceil(N / S) + S - 1
  }
  int S = 1;
  while ((long long)S * S < N) ++S;
  return S;
}

segsalsa_status make_grad_layout(const segsalsa_problem* pr, segsalsa_precision prec, int every_ck, GradLayout& gl) {
  Common c{};
  segsalsa_status s = validate_problem(pr, prec, c);
  if (s != SEGSALSA_OK) return s;
  if (every_ck < 0) return fail(SEGSALSA_ERR_INVALID_ARG, "checkpoint_every = %d < 0", every_ck);
  if (c.every > 0 || c.tol > 0.0)
    return fail(SEGSALSA_ERR_UNSUPPORTED, "the differentiable solve runs a fixed number of rounds (no residual_every/tol)");
  if (c.warm) return fail(SEGSALSA_ERR_UNSUPPORTED, "the differentiable solve starts from the input (no warm_start)");
  if (c.graph) return fail(SEGSALSA_ERR_UNSUPPORTED, "the differentiable solve launches directly (no use_graph)");
  if (c.g4s) return fail(SEGSALSA_ERR_UNSUPPORTED, "the differentiable solve uses the affine g4 (no g4_simplex)");
  if (c.pkind == kSchattenP)
    return fail(SEGSALSA_ERR_UNSUPPORTED, "the differentiable solve supports schatten_p in {1, 2, inf}");
  c.grad = 1;
  if ((s = make_batch(1, &pr->K, &pr->H, &pr->W, &pr->lambda, &pr->mu, c, gl.b)) != SEGSALSA_OK) return s;
  const Plan& p = gl.b.im[0].plan;
  gl.zbytes = align_up((size_t)p.K * p.H * p.W * p.ts);
  gl.sbytes = p.off_acc - kAccGuard - p.off_dm;
  if (every_ck == 0) every_ck = auto_interval(c.iters, gl.zbytes + gl.sbytes);
  gl.S = std::max(1, std::min(every_ck, std::max(1, c.iters)));
  gl.nck = c.iters == 0 ? 1 : ceil_div(c.iters, gl.S);
  gl.nseg = gl.S - 1;
  const size_t nt = (size_t)p.g.ntiles();
  size_t off = gl.b.total;
  gl.off_zw = off; off = align_up(off + gl.zbytes);
  gl.off_r = off; off = align_up(off + gl.zbytes);
  gl.off_bst = off; off = align_up(off + gl.sbytes);
  gl.off_pbar = off; off = align_up(off + (p.off_dm - p.off_phat));
  off += kAccGuard;
  gl.off_bacc = off; off = align_up(off + nt * (size_t)p.K * p.g.ER * p.g.EC * p.ts + kAccGuard);
  gl.off_gpart = off; off = align_up(off + nt * (size_t)(p.L + 2) * 8);
  gl.off_gtot = off; off = align_up(off + (size_t)(p.L + 2) * 8);
  gl.off_ck = off; off = align_up(off + (size_t)gl.nck * (gl.zbytes + gl.sbytes));
  gl.off_zN = off; off = align_up(off + gl.zbytes);
  gl.off_seg = off; off = align_up(off + (size_t)gl.nseg * (gl.zbytes + gl.sbytes));
  gl.total = off;
  return SEGSALSA_OK;
}

// One state (z and the multipliers) of the differentiable solve: the working
// region of the plan, or a slot (z first, then the multipliers in the plan's
// layout).
struct StateRef {
  char* z;
  char* dm;
  char* d2;
};

StateRef working_state(const GradLayout& gl, void* ws) {
  const Plan& p = gl.b.im[0].plan;
  return {wsp<char>(ws, gl.off_zw), wsp<char>(ws, p.off_dm), wsp<char>(ws, p.off_d2)};
}

StateRef slot_state(const GradLayout& gl, void* ws, size_t slot) {
  const Plan& p = gl.b.im[0].plan;
  return {wsp<char>(ws, slot), wsp<char>(ws, slot + gl.zbytes), wsp<char>(ws, slot + gl.zbytes + (p.off_d2 - p.off_dm))};
}

// The pointers of ProxArgs that name the round's input and output state, in
// declaration order (z .. d2), stored over the descriptor in one piece.
template <typename T>
struct ProxStatePtrs {
  const T* z;
  const T* phat;
  const T* dm_in;
  const T* d2_in;
  T* dm;
  T* d2;
};
static_assert(offsetof(ProxArgs<float>, acc) - offsetof(ProxArgs<float>, z) == sizeof(ProxStatePtrs<float>),
              "ProxArgs state pointers are not contiguous");
static_assert(offsetof(ProxArgs<double>, acc) - offsetof(ProxArgs<double>, z) == sizeof(ProxStatePtrs<double>),
              "ProxArgs state pointers are not contiguous");
static_assert(sizeof(ProxStatePtrs<double>) <= (size_t)kStorePairMax, "state pointers exceed one store");

// One forward round of the single image from state `in` into state `out`
// (the same region for an update in place): the round's prox descriptor
// and inverse row descriptor are pointed at the two states, then the round
// runs as usual.  No state is copied.
template <typename T>
hipError_t enqueue_round_states(const GradLayout& gl, const LaunchSet& ls, void* ws, const StateRef& in,
                                const StateRef& out, hipStream_t st) {
  const Batch& b = gl.b;
  const Plan& p = b.im[0].plan;
  ProxStatePtrs<T> sp;
  sp.z = reinterpret_cast<const T*>(in.z);
  sp.phat = wsp<T>(ws, b.im[0].base + p.off_phat);
  sp.dm_in = reinterpret_cast<const T*>(in.dm);
  sp.d2_in = reinterpret_cast<const T*>(in.d2);
  sp.dm = reinterpret_cast<T*>(out.dm);
  sp.d2 = reinterpret_cast<T*>(out.d2);
  T* zout = reinterpret_cast<T*>(out.z);
  hipError_t e = launch_store_pair(wsp<char>(ws, b.off_tab[0] + offsetof(ProxArgs<T>, z)), &sp, sizeof(sp),
                                   wsp<char>(ws, b.off_tab[4] + offsetof(RowInvArgs<T>, z)), &zout, sizeof(zout), st);
  if (e != hipSuccess) return e;
  return enqueue_round<T>(b, ls, ws, st, false);
}

template <typename T>
segsalsa_status forward_ckpt_t(const GradLayout& gl, void* ws, const void* input, void* z_out, hipStream_t st) {
  const Batch& b = gl.b;
  void* zs[1] = {wsp<char>(ws, gl.off_zw)};
  const void* ins[1] = {input};
  LaunchSet ls;
  hipError_t e = enqueue_prepare<T>(b, ws, zs, ins, st, ls, true);
  if (e != hipSuccess) return hip_fail(e, "forward set-up");
  // the initial state is the first checkpoint; every round then reads its
  // input state where the previous one wrote it and writes the next state
  // into its checkpoint slot (rounds S, 2S, ...), into zN (the last round's
  // z), or in place in the working region
  const StateRef wk = working_state(gl, ws);
  const StateRef c0 = slot_state(gl, ws, gl.ck(0));
  if ((e = launch_copy_bytes(c0.z, wk.z, gl.zbytes, st)) != hipSuccess ||
      (e = launch_copy_bytes(c0.dm, wk.dm, gl.sbytes, st)) != hipSuccess)
    return hip_fail(e, "checkpoint");
  const int N = b.c.iters;
  StateRef in = c0;
  for (int t = 0; t < N; ++t) {
    StateRef out = wk;
    if (t + 1 == N) out.z = wsp<char>(ws, gl.off_zN);
    else if ((t + 1) % gl.S == 0) out = slot_state(gl, ws, gl.ck((t + 1) / gl.S));
    if ((e = enqueue_round_states<T>(gl, ls, ws, in, out, st)) != hipSuccess) return hip_fail(e, "forward round");
    in = out;
  }
  if (N == 0 && (e = launch_copy_bytes(wsp<char>(ws, gl.off_zN), wk.z, gl.zbytes, st)) != hipSuccess)
    return hip_fail(e, "final z");
  const Plan& p = b.im[0].plan;
  if ((e = launch_copy_bytes(z_out, wsp<char>(ws, gl.off_zN), (size_t)p.K * p.H * p.W * b.c.ts, st)) != hipSuccess)
    return hip_fail(e, "z_out");
  return SEGSALSA_OK;
}

template <typename T>
segsalsa_status backward_t(const GradLayout& gl, void* ws, const void* input, const void* grad_z, void* grad_input,
                           double* grad_lambda, double* grad_weights, hipStream_t st) {
  const Batch& b = gl.b;
  const ImgRun& run = b.im[0];
  const Plan& p = run.plan;
  void* zw = wsp<char>(ws, gl.off_zw);
  void* rb = wsp<char>(ws, gl.off_r);
  void* bacc = wsp<char>(ws, gl.off_bacc);
  void* zs[1] = {zw};
  const void* ins[1] = {input};
  void* aacc[1] = {bacc};
  void* ar[1] = {rb};
  LaunchSet ls;
  hipError_t e = enqueue_prepare<T>(b, ws, zs, ins, st, ls, false, aacc, ar);
  if (e != hipSuccess) return hip_fail(e, "backward set-up");
  if ((e = launch_fill_zero(wsp<char>(ws, gl.off_bst), gl.off_bacc - gl.off_bst, st)) != hipSuccess)
    return hip_fail(e, "zero");
  if ((e = launch_fill_zero(wsp<char>(ws, gl.off_gpart), gl.off_ck - gl.off_gpart, st)) != hipSuccess)
    return hip_fail(e, "zero");
  AdjIOArgs<T> io;
  std::memset(&io, 0, sizeof(io));
  io.g = p.g;
  io.K = p.K;
  io.is_logits = b.c.logits;
  io.grad_z = reinterpret_cast<const T*>(grad_z);
  io.input = reinterpret_cast<const T*>(input);
  io.phat = wsp<T>(ws, p.off_phat);
  io.pbar = wsp<T>(ws, gl.off_pbar);
  io.acc = reinterpret_cast<T*>(bacc);
  io.frow = wsp<int>(ws, p.off_frow);
  io.fcol = wsp<int>(ws, p.off_fcol);
  io.grad_input = reinterpret_cast<T*>(grad_input);
  if ((e = launch_fill_zero(bacc, gl.off_gpart - gl.off_bacc, st)) != hipSuccess) return hip_fail(e, "zero");
  if ((e = launch_adj_load(io, st)) != hipSuccess) return hip_fail(e, "load cotangent");

  AdjArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  a.g = p.g;
  a.K = p.K;
  a.nw = p.anw;
  a.r = reinterpret_cast<const T*>(rb);
  a.phat = wsp<T>(ws, p.off_phat);
  a.bdm = wsp<T>(ws, gl.off_bst);
  a.bd2 = wsp<T>(ws, gl.off_bst + (p.off_d2 - p.off_dm));
  a.pbar = wsp<T>(ws, gl.off_pbar);
  a.acc = reinterpret_cast<T*>(bacc);
  a.gpart = wsp<double>(ws, gl.off_gpart);
  a.mu = run.mu;
  a.tau = run.lambda / run.mu;
  a.pkind = b.c.pkind;
  for (int j = 0; j < p.L; ++j) a.c[j] = (T)b.c.w[j];
  const int N = b.c.iters;
  for (int sg = gl.nck - 1; sg >= 0 && N > 0; --sg) {
    const int t0 = sg * gl.S, t1 = std::min(t0 + gl.S, N);
    // recompute the segment's states from its checkpoint, each round from
    // one slot into the next
    for (int t = t0; t + 1 < t1; ++t) {
      const StateRef in = t == t0 ? slot_state(gl, ws, gl.ck(sg)) : slot_state(gl, ws, gl.seg(t - t0 - 1));
      if ((e = enqueue_round_states<T>(gl, ls, ws, in, slot_state(gl, ws, gl.seg(t - t0)), st)) != hipSuccess)
        return hip_fail(e, "recompute");
    }
    for (int t = t1 - 1; t >= t0; --t) {
      if ((e = enqueue_fft<T>(b, ls, ws, st, 5, 6)) != hipSuccess) return hip_fail(e, "adjoint solve");
      const size_t cur = t == t0 ? gl.ck(sg) : gl.seg(t - t0 - 1);
      const size_t nxt = t + 1 < t1 ? gl.seg(t - t0) : (t1 == N ? gl.off_zN : gl.ck(sg + 1));
      a.z = wsp<T>(ws, cur);
      a.dm = wsp<T>(ws, cur + gl.zbytes);
      a.d2 = wsp<T>(ws, cur + gl.zbytes + (p.off_d2 - p.off_dm));
      a.zn = wsp<T>(ws, nxt);
      PhaseTimer t4(4, st);
      e = launch_adj_prox(a, p.g.ntiles(), p.anw * 64, p.M, p.akpw, p.adj_lds, st);
      t4.stop();
      if (e != hipSuccess) return hip_fail(e, "adjoint prox");
    }
  }
  if ((e = launch_adj_input(io, st)) != hipSuccess) return hip_fail(e, "input cotangent");
  AdjParamOut o;
  std::memset(&o, 0, sizeof(o));
  o.tot = wsp<double>(ws, gl.off_gtot);
  o.grad_weights = grad_weights;
  o.grad_lambda = grad_lambda;
  o.mu = run.mu;
  for (int j = 0; j < p.L; ++j) o.c[j] = (double)(T)b.c.w[j];
  if ((e = launch_adj_params(wsp<double>(ws, gl.off_gpart), p.g.ntiles(), p.L, o, st)) != hipSuccess)
    return hip_fail(e, "parameter cotangents");
  return SEGSALSA_OK;
}

// ---------------------------------------------------------------------------
// Autotuning: candidate launch shapes of one image shape, each timed on the
// device over a few rounds.
// ---------------------------------------------------------------------------

// Per-round milliseconds of one candidate plan: [0] whole round, [1] prox,
// [2] row DFT passes (forward and inverse), [3] column pass.
template <typename T>
hipError_t time_candidate(const Batch& b, void* ws, void* z, const void* in, hipStream_t st, int rounds,
                          double out[4]) {
  LaunchSet ls;
  void* zs[1] = {z};
  const void* ins[1] = {in};
  hipError_t e = enqueue_prepare<T>(b, ws, zs, ins, st, ls, true);
  if (e != hipSuccess) return e;
  if ((e = enqueue_round<T>(b, ls, ws, st, false)) != hipSuccess) return e;   // warm-up round
  std::vector<hipEvent_t> ev(5 * (size_t)rounds, nullptr);
  for (auto& x : ev)
    if ((e = hipEventCreate(&x)) != hipSuccess) break;
  if (e == hipSuccess)
    for (int r = 0; r < rounds && e == hipSuccess; ++r) e = enqueue_round<T>(b, ls, ws, st, false, &ev[5 * (size_t)r]);
  if (e == hipSuccess) e = hipEventSynchronize(ev.back());
  for (int q = 0; q < 4; ++q) out[q] = 0.0;
  for (int r = 0; r < rounds && e == hipSuccess; ++r) {
    float t[4];
    for (int q = 0; q < 4 && e == hipSuccess; ++q) e = hipEventElapsedTime(&t[q], ev[5 * r + q], ev[5 * r + q + 1]);
    if (e != hipSuccess) break;
    out[0] += (double)t[0] + t[1] + t[2] + t[3];
    out[1] += t[0];
    out[2] += (double)t[1] + t[3];
    out[3] += t[2];
  }
  for (auto& x : ev)
    if (x) (void)hipEventDestroy(x);
  for (int q = 0; q < 4; ++q) out[q] /= rounds;
  return e;
}

// Fill every field of a tuning record from a plan.
void tuning_of(const Plan& p, segsalsa_tuning& t) {
  t.tile_rows = p.g.TR;
  t.tile_cols = p.g.TC;
  t.classes_per_wave = p.kpw;
  t.prefetch = p.pf ? 1 : 0;
  t.col_dft = p.col_tri ? 0 : 1;
  t.generic_fft = (p.row_p2 == 0 && engine_length(p.W)) || (!p.col_tri && p.col_p2 == 0 && engine_length(p.H)) ? 1 : 0;
  t.rows_per_block = p.rows_per_block;
  t.row_threads = p.row_threads;
  t.cols_per_block = p.cols_per_block;
  t.col_threads = p.col_threads;
}

segsalsa_status check_tuning_fields(const segsalsa_tuning& t) {
  auto thr_ok = [](int v) { return v == 0 || (v >= 64 && v <= kFftMaxThreads && v % 64 == 0); };
  if (t.tile_rows < 0 || t.tile_cols < 0 || (t.tile_rows > 0) != (t.tile_cols > 0))
    return fail(SEGSALSA_ERR_INVALID_ARG, "tile %dx%d: give both sides > 0 or both 0", t.tile_rows, t.tile_cols);
  if (t.classes_per_wave != 0 && t.classes_per_wave != 1 && t.classes_per_wave != 2 && t.classes_per_wave != 4)
    return fail(SEGSALSA_ERR_INVALID_ARG, "classes_per_wave = %d (0, 1, 2 or 4)", t.classes_per_wave);
  if (t.prefetch != 0 && t.prefetch != 1) return fail(SEGSALSA_ERR_INVALID_ARG, "prefetch = %d (0 or 1)", t.prefetch);
  if (t.generic_fft != 0 && t.generic_fft != 1)
    return fail(SEGSALSA_ERR_INVALID_ARG, "generic_fft = %d (0 or 1)", t.generic_fft);
  if (t.col_dft != 0 && t.col_dft != 1) return fail(SEGSALSA_ERR_INVALID_ARG, "col_dft = %d (0 or 1)", t.col_dft);
  if (t.rows_per_block < 0 || t.cols_per_block < 0)
    return fail(SEGSALSA_ERR_INVALID_ARG, "rows/cols per block must be >= 0");
  if (!thr_ok(t.row_threads) || !thr_ok(t.col_threads))
    return fail(SEGSALSA_ERR_INVALID_ARG, "FFT threads %d / %d: 0 or a multiple of 64 in [64, %d]", t.row_threads,
                t.col_threads, kFftMaxThreads);
  if (!std::isfinite(t.us_per_round) || t.us_per_round < 0.0)
    return fail(SEGSALSA_ERR_INVALID_ARG, "us_per_round = %g", t.us_per_round);
  return SEGSALSA_OK;
}

// Parameters of a plain forward solve of one shape, for planning only.
Common plain_common(int M, segsalsa_precision prec) {
  Common c{};
  c.fp64 = prec == SEGSALSA_FP64;
  c.ts = c.fp64 ? 8 : 4;
  c.M = M;
  c.L = (2 * M + 1) * (2 * M + 1);
  for (int j = 0; j < c.L; ++j) c.w[j] = 1.0;
  c.pkind = kSchatten1;
  c.p = 1.0;
  return c;
}

segsalsa_status validate_shape(int K, int H, int W, int M, segsalsa_precision prec) {
  if (prec != SEGSALSA_FP32 && prec != SEGSALSA_FP64) return fail(SEGSALSA_ERR_INVALID_ARG, "bad precision %d", (int)prec);
  if (M < 0) return fail(SEGSALSA_ERR_INVALID_ARG, "patch_radius = %d < 0", M);
  if (M > kMaxM) return fail(SEGSALSA_ERR_UNSUPPORTED, "patch_radius = %d > %d", M, kMaxM);
  return validate_image(K, H, W, 0.0, 1.0);
}

// Minimal reader of the tuning cache: the value of "key" inside one JSON
// object's text (a number, or a string for "precision").
bool json_number(const std::string& obj, const char* key, double& v) {
  const std::string k = std::string("\"") + key + "\"";
  size_t i = obj.find(k);
  if (i == std::string::npos) return false;
  i = obj.find(':', i + k.size());
  if (i == std::string::npos) return false;
  const char* p = obj.c_str() + i + 1;
  char* end = nullptr;
  v = std::strtod(p, &end);
  return end != p;
}
bool json_string(const std::string& obj, const char* key, std::string& v) {
  const std::string k = std::string("\"") + key + "\"";
  size_t i = obj.find(k);
  if (i == std::string::npos) return false;
  i = obj.find(':', i + k.size());
  if (i == std::string::npos) return false;
  const size_t a = obj.find('"', i + 1);
  if (a == std::string::npos) return false;
  const size_t e = obj.find('"', a + 1);
  if (e == std::string::npos) return false;
  v = obj.substr(a + 1, e - a - 1);
  return true;
}

// Candidate launch shapes of the autotuner for one image shape.
std::vector<segsalsa_tuning> prox_candidates(int K, int H, int W, const Common& c) {
  std::vector<segsalsa_tuning> out;
  for (int kp : {1, 2, 4, 102}) {   // 102: two classes per wavefront, prefetching build
    const int kpw = kp % 100;
    segsalsa_tuning t{};
    t.classes_per_wave = kpw;
    t.prefetch = kp > 100 ? 1 : 0;
    Plan p;
    const std::string saved = g_last_error;
    if (plan_with(K, H, W, c, t, p) != SEGSALSA_OK) {   // this many classes per wavefront do not fit
      g_last_error = saved;
      continue;
    }
    int n = 0;
    for (const TileGeom& g : tile_candidates(p)) {
      if (!fold_lists_fit(g)) continue;
      segsalsa_tuning u = t;
      u.tile_rows = g.TR;
      u.tile_cols = g.TC;
      out.push_back(u);
      if (++n == 4) break;
    }
  }
  return out;
}

template <typename T>
segsalsa_status autotune_t(const segsalsa_problem* pr, const Common& c, const void* input, void* z, void* ws,
                           size_t wsb, int rounds, segsalsa_tuning& best, hipStream_t st) {
  const int K = pr->K, H = pr->H, W = pr->W;
  const std::string saved = g_last_error;
  // measure one candidate: false if it does not fit (plan or workspace)
  auto measure = [&](const segsalsa_tuning& tn, double out[4], segsalsa_status& err) -> bool {
    Batch b;
    err = SEGSALSA_OK;
    if (make_batch(1, &K, &H, &W, &pr->lambda, &pr->mu, c, b, &tn) != SEGSALSA_OK || b.total > wsb) {
      g_last_error = saved;
      return false;
    }
    void* zs = z;
    hipError_t e = time_candidate<T>(b, ws, zs, input, st, rounds, out);
    if (e != hipSuccess) {
      err = hip_fail(e, "autotune candidate");
      return false;
    }
    return true;
  };
  segsalsa_status err = SEGSALSA_OK;
  double t[4];
  // the planner's own choice first
  segsalsa_tuning base{};
  {
    Plan p;
    segsalsa_status s = plan_with(K, H, W, c, segsalsa_tuning{}, p);
    if (s != SEGSALSA_OK) return s;
    tuning_of(p, base);
  }
  if (!measure(base, t, err)) return err != SEGSALSA_OK ? err : fail(SEGSALSA_ERR_WORKSPACE, "workspace too small");
  const double base_round = t[0];
  segsalsa_tuning cur = base;
  double cur_round = t[0], cur_rows = t[2], cur_cols = t[3];
  // 1. prox tile and classes per wavefront, by whole rounds (the tile also sets the fold's reads)
  for (const segsalsa_tuning& pc : prox_candidates(K, H, W, c)) {
    segsalsa_tuning cand = cur;
    cand.tile_rows = pc.tile_rows;
    cand.tile_cols = pc.tile_cols;
    cand.classes_per_wave = pc.classes_per_wave;
    cand.prefetch = pc.prefetch;
    if (!measure(cand, t, err)) {
      if (err != SEGSALSA_OK) return err;
      continue;
    }
    if (t[0] < cur_round) {
      cur = cand;
      cur_round = t[0];
      cur_rows = t[2];
      cur_cols = t[3];
    }
  }
  // 2. row DFT blocking, by the two row passes
  {
    Plan p;
    if (plan_with(K, H, W, c, cur, p) != SEGSALSA_OK) return fail(SEGSALSA_ERR_DEVICE, "autotune: lost the plan");
    const int Lr = p.frow.blu ? p.frow.M : W;
    segsalsa_tuning win = cur;
    double win_t = cur_rows;
    auto consider = [&](const segsalsa_tuning& cand) -> segsalsa_status {
      if (cand.rows_per_block == cur.rows_per_block && cand.row_threads == cur.row_threads &&
          cand.generic_fft == cur.generic_fft)
        return SEGSALSA_OK;
      if (!measure(cand, t, err)) return err;
      if (t[2] < win_t) {
        win = cand;
        win_t = t[2];
      }
      return SEGSALSA_OK;
    };
    segsalsa_status s2 = SEGSALSA_OK;
    const bool pow2 = engine_length(W);
    if (pow2) {   // the fixed-structure engine: rows per workgroup (threads follow)
      for (int rpb : {1, 2, 4, 8, 16}) {
        if (rpb > H) break;
        segsalsa_tuning cand = cur;
        cand.generic_fft = 0;
        cand.rows_per_block = rpb;
        cand.row_threads = 0;
        cand.cols_per_block = cand.col_threads = 0;
        if ((s2 = consider(cand)) != SEGSALSA_OK) return s2;
      }
    }
    for (int rpb : {1, 2, 3, 4, 6, 8, 12, 16}) {   // the general kernels
      if (rpb > H) break;
      for (int per : {2, 4, 8, 16}) {
        segsalsa_tuning cand = cur;
        cand.generic_fft = pow2 ? 1 : cur.generic_fft;
        if (pow2) cand.cols_per_block = cand.col_threads = 0;
        cand.rows_per_block = rpb;
        cand.row_threads = fft_threads_for((long long)rpb * Lr, per);
        if ((s2 = consider(cand)) != SEGSALSA_OK) return s2;
      }
    }
    cur = win;
    cur_cols = 1e30;   // re-measured below with the chosen row kernels
  }
  // 3. column pass (the tridiagonal recursions or the DFTs) and its
  // blocking, by the time of the column pass
  {
    if (!measure(cur, t, err)) return err != SEGSALSA_OK ? err : fail(SEGSALSA_ERR_DEVICE, "autotune: lost the plan");
    segsalsa_tuning win = cur;
    double win_t = t[3];
    auto consider = [&](const segsalsa_tuning& cand) -> segsalsa_status {
      if (cand.cols_per_block == cur.cols_per_block && cand.col_threads == cur.col_threads &&
          cand.col_dft == cur.col_dft)
        return SEGSALSA_OK;
      if (!measure(cand, t, err)) return err;
      if (t[3] < win_t) {
        win = cand;
        win_t = t[3];
      }
      return SEGSALSA_OK;
    };
    segsalsa_status s3 = SEGSALSA_OK;
    for (int cb : {1, 2, 4, 8, 16, 32, 64}) {   // the recursions: columns per workgroup (threads follow)
      if (cb > W) break;
      segsalsa_tuning cand = cur;
      cand.col_dft = 0;
      cand.cols_per_block = cb;
      cand.col_threads = 0;
      if ((s3 = consider(cand)) != SEGSALSA_OK) return s3;
    }
    segsalsa_tuning dft = cur;
    dft.col_dft = 1;
    dft.cols_per_block = dft.col_threads = 0;
    Plan p;
    if (plan_with(K, H, W, c, dft, p) == SEGSALSA_OK) {
      const int Lc = p.fcol.blu ? p.fcol.M : H;
      if (p.col_p2) {   // the fixed-structure engine: columns per workgroup (threads follow)
        for (int cb : {1, 2, 4, 8, 16}) {
          if (cb > W) break;
          segsalsa_tuning cand = dft;
          cand.cols_per_block = cb;
          if ((s3 = consider(cand)) != SEGSALSA_OK) return s3;
        }
      } else {
        for (int cb : {1, 2, 4, 8, 16, 32}) {
          if (cb > W) break;
          for (int per : {2, 4, 8, 16}) {
            segsalsa_tuning cand = dft;
            cand.cols_per_block = cb;
            cand.col_threads = fft_threads_for((long long)cb * Lc, per);
            if ((s3 = consider(cand)) != SEGSALSA_OK) return s3;
          }
        }
      }
    } else {
      g_last_error = saved;
    }
    cur = win;
  }
  // the combination, against the planner's choice measured again
  if (!measure(cur, t, err)) return err != SEGSALSA_OK ? err : fail(SEGSALSA_ERR_DEVICE, "autotune: lost the plan");
  double tuned_round = t[0];
  if (!measure(base, t, err)) return err != SEGSALSA_OK ? err : fail(SEGSALSA_ERR_DEVICE, "autotune: lost the plan");
  const double base_again = std::min(base_round, t[0]);
  // the winner with every field filled in (threads that follow from the blocking included)
  Plan pw;
  if (plan_with(K, H, W, c, tuned_round <= base_again ? cur : base, pw) != SEGSALSA_OK)
    return fail(SEGSALSA_ERR_DEVICE, "autotune: lost the plan");
  tuning_of(pw, best);
  best.us_per_round = 1e3 * std::min(tuned_round, base_again);
  g_last_error = saved;
  return SEGSALSA_OK;
}

// Device address of `scratch` on the current GPU, looked up once per device
// (with that device current) and kept.
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;

segsalsa_status noalloc_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(SEGSALSA_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SEGSALSA_OK;
}

struct NoAllocScope {
  NoAllocScope() { g_no_alloc = true; }
  ~NoAllocScope() { g_no_alloc = false; }
};

}  // namespace

extern "C" {

const char* segsalsa_status_string(segsalsa_status s) {
  switch (s) {
    case SEGSALSA_OK: return "SEGSALSA_OK";
    case SEGSALSA_ERR_INVALID_ARG: return "SEGSALSA_ERR_INVALID_ARG";
    case SEGSALSA_ERR_UNSUPPORTED: return "SEGSALSA_ERR_UNSUPPORTED";
    case SEGSALSA_ERR_WORKSPACE: return "SEGSALSA_ERR_WORKSPACE";
    case SEGSALSA_ERR_DEVICE: return "SEGSALSA_ERR_DEVICE";
  }
  return "SEGSALSA_UNKNOWN_STATUS";
}

const char* segsalsa_last_error(void) { return g_last_error.c_str(); }

segsalsa_status segsalsa_str_workspace_size(const segsalsa_problem* prob, segsalsa_precision precision,
                                            size_t* bytes) {
  g_last_error.clear();
  if (!bytes) return fail(SEGSALSA_ERR_INVALID_ARG, "bytes is NULL");
  Batch b;
  segsalsa_status s = single_batch(prob, precision, b);
  if (s != SEGSALSA_OK) return s;
  *bytes = b.total;
  return SEGSALSA_OK;
}

segsalsa_status segsalsa_str_solve(const segsalsa_problem* prob, segsalsa_precision precision, const void* input,
                                   void* z_out, void* workspace, size_t workspace_bytes, segsalsa_stats* stats,
                                   hipStream_t stream) {
  g_last_error.clear();
  Batch b;
  segsalsa_status s = single_batch(prob, precision, b);
  if (s != SEGSALSA_OK) return s;
  const size_t ts = b.c.ts;
  if (!z_out) return fail(SEGSALSA_ERR_INVALID_ARG, "z_out is NULL");
  if (!prob->warm_start && !input) return fail(SEGSALSA_ERR_INVALID_ARG, "input is NULL");
  if (input && input == z_out) return fail(SEGSALSA_ERR_INVALID_ARG, "z_out aliases input");
  if (reinterpret_cast<uintptr_t>(z_out) % ts || reinterpret_cast<uintptr_t>(input) % ts)
    return fail(SEGSALSA_ERR_INVALID_ARG, "input/z_out not aligned to the element size");
  if ((prob->residual_every > 0 || prob->tol > 0.0) && !stats)
    return fail(SEGSALSA_ERR_INVALID_ARG, "residual_every / tol need a stats pointer");
  if ((s = check_ws(b.total, workspace, workspace_bytes)) != SEGSALSA_OK) return s;
  void* zs[1] = {z_out};
  const void* ins[1] = {input};
  return b.c.fp64 ? solve_batch_t<double>(b, workspace, zs, ins, stream, stats)
                  : solve_batch_t<float>(b, workspace, zs, ins, stream, stats);
}

segsalsa_status segsalsa_str_solve_noalloc(const segsalsa_problem* prob, segsalsa_precision precision,
                                           const void* input, void* z_out, hipStream_t stream) {
  g_last_error.clear();
  Batch b;
  segsalsa_status s = single_batch(prob, precision, b);
  if (s != SEGSALSA_OK) return s;
  if (prob->use_graph) return fail(SEGSALSA_ERR_INVALID_ARG, "the no-allocation entry point launches directly (use_graph = 0)");
  if (prob->residual_every > 0 || prob->tol > 0.0)
    return fail(SEGSALSA_ERR_INVALID_ARG, "the no-allocation entry point runs fixed rounds (residual_every = tol = 0)");
  if (b.total > (size_t)SEGSALSA_NOALLOC_SCRATCH_BYTES)
    return fail(SEGSALSA_ERR_UNSUPPORTED, "the problem needs %zu bytes of workspace, the no-allocation scratch holds %zu",
                b.total, (size_t)SEGSALSA_NOALLOC_SCRATCH_BYTES);
  const size_t ts = b.c.ts;
  if (!z_out) return fail(SEGSALSA_ERR_INVALID_ARG, "z_out is NULL");
  if (!prob->warm_start && !input) return fail(SEGSALSA_ERR_INVALID_ARG, "input is NULL");
  if (input && input == z_out) return fail(SEGSALSA_ERR_INVALID_ARG, "z_out aliases input");
  if (reinterpret_cast<uintptr_t>(z_out) % ts || reinterpret_cast<uintptr_t>(input) % ts)
    return fail(SEGSALSA_ERR_INVALID_ARG, "input/z_out not aligned to the element size");
  void* ws = nullptr;
  if ((s = noalloc_scratch(&ws)) != SEGSALSA_OK) return s;
  NoAllocScope scope;
  void* zs[1] = {z_out};
  const void* ins[1] = {input};
  return b.c.fp64 ? solve_batch_t<double>(b, ws, zs, ins, stream, nullptr)
                  : solve_batch_t<float>(b, ws, zs, ins, stream, nullptr);
}

static segsalsa_status batch_common(int32_t n, const segsalsa_image* imgs, const segsalsa_batch_params* bp,
                                    segsalsa_precision precision, Batch& b) {
  if (n < 1) return fail(SEGSALSA_ERR_INVALID_ARG, "n_images = %d < 1", n);
  if (!imgs || !bp) return fail(SEGSALSA_ERR_INVALID_ARG, "images / params is NULL");
  Common c{};
  segsalsa_status s = validate_common(bp->patch_radius, bp->patch_weights, bp->schatten_p, bp->iters,
                                      bp->input_is_logits, bp->residual_every, bp->tol, bp->warm_start, bp->use_graph,
                                      bp->g4_simplex, precision, c);
  if (s != SEGSALSA_OK) return s;
  std::vector<int> K(n), H(n), W(n);
  std::vector<double> lam(n), mu(n);
  for (int i = 0; i < n; ++i) {
    K[i] = imgs[i].K;
    H[i] = imgs[i].H;
    W[i] = imgs[i].W;
    lam[i] = imgs[i].lambda;
    mu[i] = imgs[i].mu;
  }
  s = make_batch(n, K.data(), H.data(), W.data(), lam.data(), mu.data(), c, b);
  if (s != SEGSALSA_OK) return s;
  for (int i = 0; i < n; ++i) {
    b.im[i].in_off = (size_t)imgs[i].in_offset;
    b.im[i].out_off = (size_t)imgs[i].out_offset;
    if (imgs[i].in_offset < 0 || imgs[i].out_offset < 0)
      return fail(SEGSALSA_ERR_INVALID_ARG, "image %d: negative offset", i);
  }
  return SEGSALSA_OK;
}

segsalsa_status segsalsa_str_batch_workspace_size(int32_t n_images, const segsalsa_image* images,
                                                  const segsalsa_batch_params* params, segsalsa_precision precision,
                                                  size_t* bytes) {
  g_last_error.clear();
  if (!bytes) return fail(SEGSALSA_ERR_INVALID_ARG, "bytes is NULL");
  Batch b;
  segsalsa_status s = batch_common(n_images, images, params, precision, b);
  if (s != SEGSALSA_OK) return s;
  *bytes = b.total;
  return SEGSALSA_OK;
}

segsalsa_status segsalsa_str_batch_plans(int32_t n_images, const segsalsa_image* images,
                                         const segsalsa_batch_params* params, segsalsa_precision precision,
                                         segsalsa_tuning* plans) {
  g_last_error.clear();
  if (!plans) return fail(SEGSALSA_ERR_INVALID_ARG, "plans is NULL");
  Batch b;
  segsalsa_status s = batch_common(n_images, images, params, precision, b);
  if (s != SEGSALSA_OK) return s;
  for (int i = 0; i < n_images; ++i) {
    segsalsa_tuning t{};
    tuning_of(b.im[i].plan, t);
    plans[i] = t;
  }
  return SEGSALSA_OK;
}

segsalsa_status segsalsa_str_solve_batch(int32_t n_images, const segsalsa_image* images,
                                         const segsalsa_batch_params* params, segsalsa_precision precision,
                                         const void* input_packed, void* z_packed, void* workspace,
                                         size_t workspace_bytes, segsalsa_stats* stats, hipStream_t stream) {
  g_last_error.clear();
  Batch b;
  segsalsa_status s = batch_common(n_images, images, params, precision, b);
  if (s != SEGSALSA_OK) return s;
  if (!z_packed) return fail(SEGSALSA_ERR_INVALID_ARG, "z_packed is NULL");
  if (!params->warm_start && !input_packed) return fail(SEGSALSA_ERR_INVALID_ARG, "input_packed is NULL");
  const size_t ts = b.c.ts;
  if (reinterpret_cast<uintptr_t>(z_packed) % ts || reinterpret_cast<uintptr_t>(input_packed) % ts)
    return fail(SEGSALSA_ERR_INVALID_ARG, "input/z not aligned to the element size");
  if ((params->residual_every > 0 || params->tol > 0.0) && !stats)
    return fail(SEGSALSA_ERR_INVALID_ARG, "residual_every / tol need a stats array");
  // output ranges must not overlap each other or any input range
  std::vector<std::pair<size_t, size_t>> outs;
  for (int i = 0; i < n_images; ++i) {
    const size_t nel = (size_t)images[i].K * images[i].H * images[i].W;
    outs.push_back({b.im[i].out_off, b.im[i].out_off + nel});
  }
  std::vector<std::pair<size_t, size_t>> sorted = outs;
  std::sort(sorted.begin(), sorted.end());
  for (size_t i = 1; i < sorted.size(); ++i)
    if (sorted[i].first < sorted[i - 1].second) return fail(SEGSALSA_ERR_INVALID_ARG, "output ranges overlap");
  if (input_packed == z_packed) return fail(SEGSALSA_ERR_INVALID_ARG, "z_packed aliases input_packed");
  if ((s = check_ws(b.total, workspace, workspace_bytes)) != SEGSALSA_OK) return s;
  std::vector<void*> zs(n_images);
  std::vector<const void*> ins(n_images);
  for (int i = 0; i < n_images; ++i) {
    zs[i] = reinterpret_cast<char*>(z_packed) + b.im[i].out_off * ts;
    ins[i] = input_packed ? reinterpret_cast<const char*>(input_packed) + b.im[i].in_off * ts : nullptr;
  }
  return b.c.fp64 ? solve_batch_t<double>(b, workspace, zs.data(), ins.data(), stream, stats)
                  : solve_batch_t<float>(b, workspace, zs.data(), ins.data(), stream, stats);
}

segsalsa_status segsalsa_str_labels(int32_t K, int32_t H, int32_t W, segsalsa_precision precision, const void* z,
                                    int32_t* labels, hipStream_t stream) {
  g_last_error.clear();
  if (K < 1 || H < 1 || W < 1) return fail(SEGSALSA_ERR_INVALID_ARG, "bad shape K=%d H=%d W=%d", K, H, W);
  if (!z || !labels) return fail(SEGSALSA_ERR_INVALID_ARG, "NULL pointer");
  if (precision != SEGSALSA_FP32 && precision != SEGSALSA_FP64) return fail(SEGSALSA_ERR_INVALID_ARG, "bad precision");
  hipError_t e = precision == SEGSALSA_FP64
                     ? launch_labels(K, H, W, reinterpret_cast<const double*>(z), labels, stream)
                     : launch_labels(K, H, W, reinterpret_cast<const float*>(z), labels, stream);
  return e == hipSuccess ? SEGSALSA_OK : hip_fail(e, "labels kernel");
}

segsalsa_status segsalsa_str_state_export(const segsalsa_problem* prob, segsalsa_precision precision,
                                          const void* workspace, size_t workspace_bytes, void* d1, void* d2, void* d3,
                                          void* d4, hipStream_t stream) {
  g_last_error.clear();
  Batch b;
  segsalsa_status s = single_batch(prob, precision, b);
  if (s != SEGSALSA_OK) return s;
  if ((s = check_ws(b.total, workspace, workspace_bytes)) != SEGSALSA_OK) return s;
  void* ws = const_cast<void*>(workspace);
  const Plan& p = b.im[0].plan;
  hipError_t e = p.fp64 ? run_state<double>(p, ws, 1, nullptr, d1, d2, d3, d4, stream)
                        : run_state<float>(p, ws, 1, nullptr, d1, d2, d3, d4, stream);
  return e == hipSuccess ? SEGSALSA_OK : hip_fail(e, "state export kernel");
}

segsalsa_status segsalsa_str_state_import(const segsalsa_problem* prob, segsalsa_precision precision, void* workspace,
                                          size_t workspace_bytes, const void* p_hat, const void* d1, const void* d2,
                                          const void* d3, const void* d4, hipStream_t stream) {
  g_last_error.clear();
  Batch b;
  segsalsa_status s = single_batch(prob, precision, b);
  if (s != SEGSALSA_OK) return s;
  if ((s = check_ws(b.total, workspace, workspace_bytes)) != SEGSALSA_OK) return s;
  if (!p_hat || !d1 || !d2 || !d3 || !d4) return fail(SEGSALSA_ERR_INVALID_ARG, "state import needs all arrays");
  const Plan& p = b.im[0].plan;
  hipError_t e = p.fp64 ? run_state<double>(p, workspace, 0, p_hat, d1, d2, d3, d4, stream)
                        : run_state<float>(p, workspace, 0, p_hat, d1, d2, d3, d4, stream);
  return e == hipSuccess ? SEGSALSA_OK : hip_fail(e, "state import kernel");
}

segsalsa_status segsalsa_str_grad_workspace_size(const segsalsa_problem* prob, segsalsa_precision precision,
                                                 int32_t checkpoint_every, size_t* bytes) {
  g_last_error.clear();
  if (!bytes) return fail(SEGSALSA_ERR_INVALID_ARG, "bytes is NULL");
  GradLayout gl;
  segsalsa_status s = make_grad_layout(prob, precision, checkpoint_every, gl);
  if (s != SEGSALSA_OK) return s;
  *bytes = gl.total;
  return SEGSALSA_OK;
}

segsalsa_status segsalsa_str_grad_checkpoint_interval(const segsalsa_problem* prob, segsalsa_precision precision,
                                                      int32_t checkpoint_every, int32_t* interval) {
  g_last_error.clear();
  if (!interval) return fail(SEGSALSA_ERR_INVALID_ARG, "interval is NULL");
  GradLayout gl;
  segsalsa_status s = make_grad_layout(prob, precision, checkpoint_every, gl);
  if (s != SEGSALSA_OK) return s;
  *interval = gl.S;
  return SEGSALSA_OK;
}

segsalsa_status segsalsa_str_solve_ckpt(const segsalsa_problem* prob, segsalsa_precision precision,
                                        int32_t checkpoint_every, const void* input, void* z_out, void* workspace,
                                        size_t workspace_bytes, hipStream_t stream) {
  g_last_error.clear();
  GradLayout gl;
  segsalsa_status s = make_grad_layout(prob, precision, checkpoint_every, gl);
  if (s != SEGSALSA_OK) return s;
  const size_t ts = gl.b.c.ts;
  if (!input || !z_out) return fail(SEGSALSA_ERR_INVALID_ARG, "input / z_out is NULL");
  if (input == z_out) return fail(SEGSALSA_ERR_INVALID_ARG, "z_out aliases input");
  if (reinterpret_cast<uintptr_t>(z_out) % ts || reinterpret_cast<uintptr_t>(input) % ts)
    return fail(SEGSALSA_ERR_INVALID_ARG, "input/z_out not aligned to the element size");
  if ((s = check_ws(gl.total, workspace, workspace_bytes)) != SEGSALSA_OK) return s;
  return gl.b.c.fp64 ? forward_ckpt_t<double>(gl, workspace, input, z_out, stream)
                     : forward_ckpt_t<float>(gl, workspace, input, z_out, stream);
}

segsalsa_status segsalsa_str_backward(const segsalsa_problem* prob, segsalsa_precision precision,
                                      int32_t checkpoint_every, const void* input, const void* grad_z,
                                      void* grad_input, double* grad_lambda, double* grad_weights, void* workspace,
                                      size_t workspace_bytes, hipStream_t stream) {
  g_last_error.clear();
  GradLayout gl;
  segsalsa_status s = make_grad_layout(prob, precision, checkpoint_every, gl);
  if (s != SEGSALSA_OK) return s;
  const size_t ts = gl.b.c.ts;
  if (!input || !grad_z || !grad_input) return fail(SEGSALSA_ERR_INVALID_ARG, "input / grad_z / grad_input is NULL");
  if (grad_input == input || grad_input == grad_z)
    return fail(SEGSALSA_ERR_INVALID_ARG, "grad_input aliases input or grad_z");
  if (reinterpret_cast<uintptr_t>(input) % ts || reinterpret_cast<uintptr_t>(grad_z) % ts ||
      reinterpret_cast<uintptr_t>(grad_input) % ts)
    return fail(SEGSALSA_ERR_INVALID_ARG, "arrays not aligned to the element size");
  if (reinterpret_cast<uintptr_t>(grad_lambda) % 8 || reinterpret_cast<uintptr_t>(grad_weights) % 8)
    return fail(SEGSALSA_ERR_INVALID_ARG, "grad_lambda / grad_weights not 8-byte aligned");
  if ((s = check_ws(gl.total, workspace, workspace_bytes)) != SEGSALSA_OK) return s;
  return gl.b.c.fp64 ? backward_t<double>(gl, workspace, input, grad_z, grad_input, grad_lambda, grad_weights, stream)
                     : backward_t<float>(gl, workspace, input, grad_z, grad_input, grad_lambda, grad_weights, stream);
}

segsalsa_status segsalsa_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t stream) {
  g_last_error.clear();
  if (bytes == 0) return SEGSALSA_OK;
  if (!src || !dst) return fail(SEGSALSA_ERR_INVALID_ARG, "stream copy: NULL pointer");
  if (bytes % 16 != 0 || reinterpret_cast<uintptr_t>(src) % 16 != 0 || reinterpret_cast<uintptr_t>(dst) % 16 != 0)
    return fail(SEGSALSA_ERR_INVALID_ARG, "stream copy: pointers and size must be multiples of 16 bytes");
  const uintptr_t s0 = reinterpret_cast<uintptr_t>(src), d0 = reinterpret_cast<uintptr_t>(dst);
  if (s0 < d0 + bytes && d0 < s0 + bytes) return fail(SEGSALSA_ERR_INVALID_ARG, "stream copy: buffers overlap");
  const hipError_t e = launch_stream_copy(dst, src, bytes, stream);
  return e == hipSuccess ? SEGSALSA_OK : hip_fail(e, "stream copy");
}

segsalsa_status segsalsa_profile_enable(int32_t on) {
  g_last_error.clear();
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.on = on != 0;
  return SEGSALSA_OK;
}

segsalsa_status segsalsa_profile_read(double* ms, int64_t* launches, int32_t reset) {
  g_last_error.clear();
  std::lock_guard<std::mutex> lk(g_prof.mu);
  for (auto& pe : g_prof.pending) {
    float t = 0.0f;
    hipError_t e = hipEventSynchronize(pe.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, pe.a, pe.b);
    if (e != hipSuccess) return hip_fail(e, "profile event");
    g_prof.ms[pe.phase] += t;
    g_prof.count[pe.phase] += 1;
    g_prof.pool.push_back(pe.a);
    g_prof.pool.push_back(pe.b);
  }
  g_prof.pending.clear();
  for (int i = 0; i < SEGSALSA_NUM_PHASES; ++i) {
    if (ms) ms[i] = g_prof.ms[i];
    if (launches) launches[i] = g_prof.count[i];
    if (reset) {
      g_prof.ms[i] = 0.0;
      g_prof.count[i] = 0;
    }
  }
  return SEGSALSA_OK;
}


segsalsa_status segsalsa_tuning_set(int32_t K, int32_t H, int32_t W, int32_t patch_radius,
                                    segsalsa_precision precision, const segsalsa_tuning* tuning) {
  g_last_error.clear();
  segsalsa_status s = validate_shape(K, H, W, patch_radius, precision);
  if (s != SEGSALSA_OK) return s;
  const TuneKey key{K, H, W, patch_radius, precision == SEGSALSA_FP64 ? 1 : 0};
  if (!tuning) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.erase(key);
    return SEGSALSA_OK;
  }
  if ((s = check_tuning_fields(*tuning)) != SEGSALSA_OK) return s;
  Plan p;
  if ((s = plan_with(K, H, W, plain_common(patch_radius, precision), *tuning, p)) != SEGSALSA_OK) return s;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = *tuning;
  return SEGSALSA_OK;
}

segsalsa_status segsalsa_tuning_get(int32_t K, int32_t H, int32_t W, int32_t patch_radius,
                                    segsalsa_precision precision, segsalsa_tuning* out, int32_t* tuned) {
  g_last_error.clear();
  if (!out) return fail(SEGSALSA_ERR_INVALID_ARG, "out is NULL");
  segsalsa_status s = validate_shape(K, H, W, patch_radius, precision);
  if (s != SEGSALSA_OK) return s;
  Plan p;
  if ((s = make_image_plan(K, H, W, plain_common(patch_radius, precision), p)) != SEGSALSA_OK) return s;
  segsalsa_tuning t{};
  tuning_of(p, t);
  segsalsa_tuning ent{};
  if (p.tuned && tuning_lookup(K, H, W, patch_radius, precision == SEGSALSA_FP64, ent)) t.us_per_round = ent.us_per_round;
  *out = t;
  if (tuned) *tuned = p.tuned ? 1 : 0;
  return SEGSALSA_OK;
}

segsalsa_status segsalsa_tuning_clear(void) {
  g_last_error.clear();
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  return SEGSALSA_OK;
}

segsalsa_status segsalsa_tuning_save(const char* path) {
  g_last_error.clear();
  if (!path) return fail(SEGSALSA_ERR_INVALID_ARG, "path is NULL");
  std::string txt = "{\n  \"format\": \"segsalsa-tuning-1\",\n  \"entries\": [";
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    bool first = true;
    for (const auto& kv : g_tune) {
      const TuneKey& k = kv.first;
      const segsalsa_tuning& t = kv.second;
      char buf[512];
      std::snprintf(buf, sizeof(buf),
                    "%s\n    {\"K\": %d, \"H\": %d, \"W\": %d, \"M\": %d, \"precision\": \"%s\", \"tile_rows\": %d, "
                    "\"tile_cols\": %d, \"classes_per_wave\": %d, \"prefetch\": %d, \"generic_fft\": %d, "
                    "\"col_dft\": %d, \"rows_per_block\": %d, \"row_threads\": %d, \"cols_per_block\": %d, "
                    "\"col_threads\": %d, \"us_per_round\": %.3f}",
                    first ? "" : ",", k.K, k.H, k.W, k.M, k.fp64 ? "fp64" : "fp32", t.tile_rows, t.tile_cols,
                    t.classes_per_wave, t.prefetch, t.generic_fft, t.col_dft, t.rows_per_block, t.row_threads,
                    t.cols_per_block, t.col_threads, t.us_per_round);
      txt += buf;
      first = false;
    }
  }
  txt += "\n  ]\n}\n";
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(SEGSALSA_ERR_INVALID_ARG, "cannot write %s", path);
  const bool ok = std::fwrite(txt.data(), 1, txt.size(), f) == txt.size();
  if (std::fclose(f) != 0 || !ok) return fail(SEGSALSA_ERR_INVALID_ARG, "cannot write %s", path);
  return SEGSALSA_OK;
}

segsalsa_status segsalsa_tuning_load(const char* path, int32_t* loaded, int32_t* skipped) {
  g_last_error.clear();
  if (loaded) *loaded = 0;
  if (skipped) *skipped = 0;
  if (!path) return fail(SEGSALSA_ERR_INVALID_ARG, "path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(SEGSALSA_ERR_INVALID_ARG, "cannot read %s", path);
  std::string txt;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, n);
  std::fclose(f);
  std::string fmt;
  if (!json_string(txt, "format", fmt) || fmt != "segsalsa-tuning-1")
    return fail(SEGSALSA_ERR_INVALID_ARG, "%s is not a segsalsa tuning cache", path);
  size_t pos = txt.find("\"entries\"");
  if (pos == std::string::npos) return fail(SEGSALSA_ERR_INVALID_ARG, "%s has no entries", path);
  int nl = 0, ns = 0;
  while ((pos = txt.find('{', pos)) != std::string::npos) {
    const size_t end = txt.find('}', pos);
    if (end == std::string::npos) break;
    const std::string obj = txt.substr(pos, end - pos + 1);
    pos = end + 1;
    double K, H, W, M, tr, tc, kpw, rpb, rt, cpb, ct, us = 0.0, pf = 0.0, gf = 0.0, cd = 0.0;
    std::string prec;
    if (!(json_number(obj, "K", K) && json_number(obj, "H", H) && json_number(obj, "W", W) &&
          json_number(obj, "M", M) && json_string(obj, "precision", prec) && json_number(obj, "tile_rows", tr) &&
          json_number(obj, "tile_cols", tc) && json_number(obj, "classes_per_wave", kpw) &&
          json_number(obj, "rows_per_block", rpb) && json_number(obj, "row_threads", rt) &&
          json_number(obj, "cols_per_block", cpb) && json_number(obj, "col_threads", ct)) ||
        (prec != "fp32" && prec != "fp64")) {
      ++ns;
      continue;
    }
    (void)json_number(obj, "us_per_round", us);
    (void)json_number(obj, "prefetch", pf);
    (void)json_number(obj, "generic_fft", gf);
    (void)json_number(obj, "col_dft", cd);
    segsalsa_tuning t{};
    t.tile_rows = (int)tr; t.tile_cols = (int)tc; t.classes_per_wave = (int)kpw; t.prefetch = (int)pf;
    t.generic_fft = (int)gf;
    t.col_dft = (int)cd;
    t.rows_per_block = (int)rpb; t.row_threads = (int)rt; t.cols_per_block = (int)cpb; t.col_threads = (int)ct;
    t.us_per_round = us;
    if (segsalsa_tuning_set((int)K, (int)H, (int)W, (int)M, prec == "fp64" ? SEGSALSA_FP64 : SEGSALSA_FP32, &t) ==
        SEGSALSA_OK)
      ++nl;
    else
      ++ns;
  }
  g_last_error.clear();
  if (loaded) *loaded = nl;
  if (skipped) *skipped = ns;
  return SEGSALSA_OK;
}

segsalsa_status segsalsa_str_autotune_workspace_size(const segsalsa_problem* prob, segsalsa_precision precision,
                                                     size_t* bytes) {
  g_last_error.clear();
  if (!bytes) return fail(SEGSALSA_ERR_INVALID_ARG, "bytes is NULL");
  Common c{};
  segsalsa_status s = validate_problem(prob, precision, c);
  if (s != SEGSALSA_OK) return s;
  c.every = 0; c.tol = 0.0; c.warm = 0; c.graph = 0;
  size_t best = 0;
  std::vector<segsalsa_tuning> cands = prox_candidates(prob->K, prob->H, prob->W, c);
  cands.push_back(segsalsa_tuning{});
  for (const segsalsa_tuning& t : cands) {
    Batch b;
    if (make_batch(1, &prob->K, &prob->H, &prob->W, &prob->lambda, &prob->mu, c, b, &t) == SEGSALSA_OK)
      best = std::max(best, b.total);
  }
  g_last_error.clear();
  if (best == 0) return fail(SEGSALSA_ERR_UNSUPPORTED, "no launch shape fits this problem");
  *bytes = best;
  return SEGSALSA_OK;
}

segsalsa_status segsalsa_str_autotune(const segsalsa_problem* prob, segsalsa_precision precision,
                                      const void* input, void* z_scratch, void* workspace, size_t workspace_bytes,
                                      int32_t rounds, segsalsa_tuning* best, hipStream_t stream) {
  g_last_error.clear();
  Common c{};
  segsalsa_status s = validate_problem(prob, precision, c);
  if (s != SEGSALSA_OK) return s;
  if (rounds < 1 || rounds > 100) return fail(SEGSALSA_ERR_INVALID_ARG, "rounds = %d not in [1, 100]", rounds);
  if (!input || !z_scratch) return fail(SEGSALSA_ERR_INVALID_ARG, "input / z_scratch is NULL");
  if (input == z_scratch) return fail(SEGSALSA_ERR_INVALID_ARG, "z_scratch aliases input");
  if (reinterpret_cast<uintptr_t>(z_scratch) % c.ts || reinterpret_cast<uintptr_t>(input) % c.ts)
    return fail(SEGSALSA_ERR_INVALID_ARG, "input/z_scratch not aligned to the element size");
  if ((s = check_ws(1, workspace, workspace_bytes)) != SEGSALSA_OK) return s;
  c.every = 0; c.tol = 0.0; c.warm = 0; c.graph = 0;
  segsalsa_tuning win{};
  s = c.fp64 ? autotune_t<double>(prob, c, input, z_scratch, workspace, workspace_bytes, rounds, win, stream)
             : autotune_t<float>(prob, c, input, z_scratch, workspace, workspace_bytes, rounds, win, stream);
  if (s != SEGSALSA_OK) return s;
  if ((s = segsalsa_tuning_set(prob->K, prob->H, prob->W, prob->patch_radius, precision, &win)) != SEGSALSA_OK)
    return s;
  if (best) *best = win;
  return SEGSALSA_OK;
}

}  // extern "C"
