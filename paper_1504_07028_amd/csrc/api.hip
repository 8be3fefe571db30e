// Host runtime of the SegSALSA-STR C ABI: argument validation, plan (tile
// grid, FFT factorisations, workspace layout) and the per-round launch
// sequence.  See include/segsalsa.h for the contract of each entry point.
#include "segsalsa.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "segsalsa_internal.h"
#include "segsalsa_kernels.h"

using namespace segsalsa;

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

FftPlanDev make_fft_plan(int N) {
  FftPlanDev p;
  std::memset(&p, 0, sizeof(p));
  p.N = N;
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
  p.nst = (int)r.size();
  for (int i = 0; i < p.nst; ++i) p.rad[i] = r[i];
  return p;
}

struct Plan {
  bool fp64;
  size_t ts;     // sizeof(T)
  int K, H, W, M, L, P;
  TileGeom g;
  int nw, kpw;   // prox workgroup: wavefronts and classes per wavefront
  size_t prox_lds;
  FftPlanDev frow, fcol;
  int rows_per_block, row_threads, row_ept;
  size_t row_lds;
  int cols_per_block, col_threads, col_ept;
  size_t col_lds;
  // workspace offsets (bytes)
  size_t off_flags, off_twW, off_twH, off_sx, off_sy, off_frow, off_fcol, off_phat, off_dm, off_d2, off_acc, off_spec,
      off_zprev, off_restile, off_partial, off_out, total;
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
    if (fold_list(g, r, true, nullptr) < 0) return false;
  for (int c = 0; c < g.W; ++c)
    if (fold_list(g, c, false, nullptr) < 0) return false;
  return true;
}

// Tile grid of the prox kernel.  A workgroup processes one tile in
// ceil(pixels / 64) steps plus a fixed load/store phase; tiles run in
// batches of (compute units x resident workgroups).  Among the shapes whose
// LDS footprint fits, take the one with the fewest batches x (steps + 1),
// breaking ties by the smaller grown-tile overhead.  SEGSALSA_TILE=RxC forces
// a shape (tuning runs).
bool choose_tiles(Plan& p) {
  static const int rows[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16};
  static const int cols[] = {8, 12, 16, 20, 24, 32, 40, 48, 64};
  const size_t part = 12 * (size_t)p.nw * 64;
  auto lds_of = [&](const TileGeom& g) { return (2 * (size_t)p.K * g.ER * g.EC + part) * p.ts + 16; };
  // resident workgroups per CU allowed by the register budget of the chosen instantiation
  const int waves_per_simd = std::max(1, prox_max_threads_rt(p.fp64, p.M, p.kpw) / 256);
  const int occ_regs = std::max(1, (4 * waves_per_simd) / p.nw);
  const char* env = std::getenv("SEGSALSA_TILE");
  int fr = 0, fc = 0;
  if (env && std::sscanf(env, "%dx%d", &fr, &fc) == 2 && fr > 0 && fc > 0) {
    TileGeom g = tile_geom(p, fr, fc);
    if (lds_of(g) <= kLdsBudget && fold_lists_fit(g)) {
      p.g = g;
      p.prox_lds = lds_of(g);
      return true;
    }
  }
  bool have = false;
  TileGeom best{};
  double best_cost = 0, best_over = 0;
  for (int tr : rows) {
    for (int tc : cols) {
      TileGeom g = tile_geom(p, tr, tc);
      const size_t lds = lds_of(g);
      if (lds > kLdsBudget) continue;
      const int occ = std::max(1, std::min(occ_regs, (int)(kLdsBudget / lds)));
      const long long slots = (long long)kTargetGroups * occ;
      const long long batches = (g.ntiles() + slots - 1) / slots;
      const double cost = (double)batches * (g.steps + 1);
      const double over = (double)g.ER * g.EC / ((double)g.TR * g.TC);
      if (!have || cost < best_cost || (cost == best_cost && over < best_over)) {
        if (!fold_lists_fit(g)) continue;
        have = true;
        best = g;
        best_cost = cost;
        best_over = over;
      }
    }
  }
  if (!have) return false;
  p.g = best;
  p.prox_lds = lds_of(best);
  return true;
}

// Elements per thread (2, 4, 8 or 16) and workgroup size of an LDS FFT
// workgroup holding `items` complex elements: the fewest elements per thread
// that keep the workgroup within 1024 threads.
void fft_threads(long long items, int& ept, int& threads) {
  ept = 2;
  while (ept < kFftEptMax && (items + ept - 1) / ept > 1024) ept *= 2;
  long long t = (items + ept - 1) / ept;
  t = (t + 63) / 64 * 64;
  threads = (int)std::max<long long>(64, std::min<long long>(t, 1024));
}

segsalsa_status validate(const segsalsa_problem* pr, segsalsa_precision prec) {
  if (!pr) return fail(SEGSALSA_ERR_INVALID_ARG, "problem is NULL");
  if (prec != SEGSALSA_FP32 && prec != SEGSALSA_FP64) return fail(SEGSALSA_ERR_INVALID_ARG, "bad precision %d", (int)prec);
  if (pr->K < 2) return fail(SEGSALSA_ERR_INVALID_ARG, "K = %d must be >= 2", pr->K);
  if (pr->K > kMaxK) return fail(SEGSALSA_ERR_UNSUPPORTED, "K = %d exceeds %d", pr->K, kMaxK);
  if (pr->H < 1 || pr->W < 1) return fail(SEGSALSA_ERR_INVALID_ARG, "H = %d, W = %d must be >= 1", pr->H, pr->W);
  if ((long long)pr->H * pr->W < 2) return fail(SEGSALSA_ERR_INVALID_ARG, "image must have >= 2 pixels");
  if (pr->H > kMaxSide || pr->W > kMaxSide)
    return fail(SEGSALSA_ERR_UNSUPPORTED, "H = %d, W = %d exceed %d", pr->H, pr->W, kMaxSide);
  if (pr->patch_radius < 0) return fail(SEGSALSA_ERR_INVALID_ARG, "patch_radius = %d < 0", pr->patch_radius);
  if (pr->patch_radius > kMaxM) return fail(SEGSALSA_ERR_UNSUPPORTED, "patch_radius = %d > %d", pr->patch_radius, kMaxM);
  if (!pr->patch_weights) return fail(SEGSALSA_ERR_INVALID_ARG, "patch_weights is NULL");
  const int L = (2 * pr->patch_radius + 1) * (2 * pr->patch_radius + 1);
  for (int j = 0; j < L; ++j)
    if (!std::isfinite(pr->patch_weights[j])) return fail(SEGSALSA_ERR_INVALID_ARG, "patch weight %d not finite", j);
  const double p = pr->schatten_p;
  if (std::isnan(p)) return fail(SEGSALSA_ERR_INVALID_ARG, "schatten_p is NaN");
  if (!(p == 1.0 || p == 2.0 || (std::isinf(p) && p > 0)))
    return fail(SEGSALSA_ERR_UNSUPPORTED, "schatten_p = %g (supported: 1, 2, inf)", p);
  if (!std::isfinite(pr->lambda) || pr->lambda < 0.0) return fail(SEGSALSA_ERR_INVALID_ARG, "lambda = %g", pr->lambda);
  if (!std::isfinite(pr->mu) || !(pr->mu > 0.0)) return fail(SEGSALSA_ERR_INVALID_ARG, "mu = %g", pr->mu);
  if (pr->iters < 0) return fail(SEGSALSA_ERR_INVALID_ARG, "iters = %d < 0", pr->iters);
  if (pr->input_is_logits != 0 && pr->input_is_logits != 1)
    return fail(SEGSALSA_ERR_INVALID_ARG, "input_is_logits = %d", pr->input_is_logits);
  if (pr->residual_every < 0) return fail(SEGSALSA_ERR_INVALID_ARG, "residual_every = %d", pr->residual_every);
  if (!std::isfinite(pr->tol) || pr->tol < 0.0) return fail(SEGSALSA_ERR_INVALID_ARG, "tol = %g", pr->tol);
  if (pr->tol > 0.0 && pr->residual_every == 0)
    return fail(SEGSALSA_ERR_INVALID_ARG, "tol > 0 needs residual_every > 0");
  if (pr->warm_start != 0 && pr->warm_start != 1)
    return fail(SEGSALSA_ERR_INVALID_ARG, "warm_start = %d", pr->warm_start);
  return SEGSALSA_OK;
}

segsalsa_status make_plan(const segsalsa_problem* pr, segsalsa_precision prec, Plan& p) {
  segsalsa_status s = validate(pr, prec);
  if (s != SEGSALSA_OK) return s;
  p.fp64 = prec == SEGSALSA_FP64;
  p.ts = p.fp64 ? 8 : 4;
  p.K = pr->K; p.H = pr->H; p.W = pr->W; p.M = pr->patch_radius;
  p.L = (2 * p.M + 1) * (2 * p.M + 1);
  p.P = (p.K + 1) / 2;
  // prox workgroup: fewest classes per wavefront whose register budget allows ceil(K/kpw) wavefronts
  p.kpw = 0;
  int kpw_first = 1;
  if (const char* ek = std::getenv("SEGSALSA_KPW")) kpw_first = std::atoi(ek);
  for (int kpw : {1, 2, 4}) {
    if (kpw < kpw_first) continue;
    const int nw = ceil_div(p.K, kpw);
    if (nw <= 16 && nw * 64 <= prox_max_threads_rt(p.fp64, p.M, kpw)) {
      p.kpw = kpw;
      p.nw = nw;
      break;
    }
  }
  if (p.kpw == 0) {
    p.kpw = 4;
    p.nw = ceil_div(p.K, 4);
    if (p.nw * 64 > prox_max_threads_rt(p.fp64, p.M, 4))
      return fail(SEGSALSA_ERR_UNSUPPORTED, "K = %d, M = %d do not fit one workgroup", p.K, p.M);
  }
  if (!choose_tiles(p)) return fail(SEGSALSA_ERR_UNSUPPORTED, "no tile shape fits LDS for K = %d, M = %d", p.K, p.M);
  // FFT passes
  const size_t cs = 2 * p.ts;
  p.frow = make_fft_plan(p.W);
  p.fcol = make_fft_plan(p.H);
  // FFT workgroups: a few hundred elements per workgroup at one or two per
  // thread for latency hiding, whole rows (columns) plus the twiddle table in
  // LDS; column blocks of 8+ columns on tall images for coalesced rows.
  const long long cap = p.fp64 ? 6144 : 12288;   // complex elements per FFT workgroup
  {
    long long rpb = std::max<long long>(1, 512 / p.W);
    rpb = std::max<long long>(1, std::min<long long>(rpb, p.H));
    p.rows_per_block = (int)rpb;
    fft_threads(rpb * p.W, p.row_ept, p.row_threads);
    p.row_lds = (size_t)(rpb + 1) * p.W * cs;
  }
  {
    int cb = 1;
    while (cb < 64 && cb * 2 <= p.W && (long long)(cb * 2) * p.H <= cap &&
           ((long long)(cb * 2) * p.H <= 1024 || cb * 2 <= 8))
      cb *= 2;
    p.cols_per_block = cb;
    fft_threads((long long)cb * p.H, p.col_ept, p.col_threads);
    p.col_lds = (size_t)(cb + 1) * p.H * cs;
  }
  // workspace layout
  const size_t nt = (size_t)p.g.ntiles();
  size_t off = 0;
  p.off_flags = off; off = align_up(off + 64);
  p.off_twW = off; off = align_up(off + (size_t)p.W * cs);
  p.off_twH = off; off = align_up(off + (size_t)p.H * cs);
  p.off_sx = off; off = align_up(off + (size_t)p.W * 8);
  p.off_sy = off; off = align_up(off + (size_t)p.H * 8);
  p.off_frow = off; off = align_up(off + (size_t)p.H * kFoldStride * 4);
  p.off_fcol = off; off = align_up(off + (size_t)p.W * kFoldStride * 4);
  const size_t per_step = (size_t)p.K * 64 * p.ts;
  p.off_phat = off; off = align_up(off + nt * p.g.steps * per_step);
  p.off_dm = off; off = align_up(off + nt * p.g.steps * per_step * 3);
  p.off_d2 = off; off = align_up(off + nt * p.g.steps * per_step * 2 * p.L);
  p.off_acc = off; off = align_up(off + nt * (size_t)p.K * p.g.ER * p.g.EC * p.ts);
  p.off_spec = off; off = align_up(off + (size_t)p.P * p.H * p.W * cs);
  // convergence diagnostics
  p.off_zprev = off; off = align_up(off + (size_t)p.K * p.H * p.W * p.ts);
  p.off_restile = off; off = align_up(off + nt * 8);
  p.npartial = std::max<int>(kDiagBlocks, (int)(((size_t)p.H * p.W + 255) / 256));
  p.off_partial = off; off = align_up(off + (size_t)p.npartial * 8);
  p.off_out = off; off = align_up(off + 4 * 8);
  p.total = off;
  if (const char* lg = std::getenv("SEGSALSA_LOG")) {
    if (lg[0] == '1')
      std::fprintf(stderr,
                   "[segsalsa] plan %s K=%d H=%d W=%d M=%d: tiles %dx%d (max %dx%d, %d tiles, %d steps), prox nw=%d "
                   "kpw=%d lds=%zu; rows/block=%d threads=%d ept=%d; cols/block=%d threads=%d ept=%d; workspace %zu B\n",
                   p.fp64 ? "fp64" : "fp32", p.K, p.H, p.W, p.M, p.g.ntr, p.g.ntc, p.g.TR, p.g.TC, p.g.ntiles(),
                   p.g.steps, p.nw, p.kpw, p.prox_lds, p.rows_per_block, p.row_threads, p.row_ept, p.cols_per_block,
                   p.col_threads, p.col_ept, p.total);
  }
  return SEGSALSA_OK;
}

template <typename T>
T* wsp(void* ws, size_t off) { return reinterpret_cast<T*>(reinterpret_cast<char*>(ws) + off); }

segsalsa_status check_ws(const Plan& p, const void* ws, size_t bytes) {
  if (!ws) return fail(SEGSALSA_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(SEGSALSA_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (bytes < p.total) return fail(SEGSALSA_ERR_WORKSPACE, "workspace %zu bytes < required %zu", bytes, p.total);
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

struct PhaseTimer {
  int phase;
  hipStream_t st;
  hipEvent_t a = nullptr;
  PhaseTimer(int ph, hipStream_t s) : phase(ph), st(s) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    if (!g_prof.on) return;
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

template <typename T>
hipError_t enqueue_round(const Plan& p, const segsalsa_problem* pr, T* z, void* ws, hipStream_t st,
                         bool residuals = false) {
  ProxArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  a.g = p.g;
  a.K = p.K;
  a.nw = p.nw;
  a.z = z;
  a.phat = wsp<T>(ws, p.off_phat);
  a.dm = wsp<T>(ws, p.off_dm);
  a.d2 = wsp<T>(ws, p.off_d2);
  a.acc = wsp<T>(ws, p.off_acc);
  a.res_tile = residuals ? wsp<double>(ws, p.off_restile) : nullptr;
  a.mu = pr->mu;
  a.tau = pr->lambda / pr->mu;
  a.pkind = pr->schatten_p == 1.0 ? kSchatten1 : (pr->schatten_p == 2.0 ? kSchatten2 : kSchattenInf);
  for (int j = 0; j < p.L; ++j) a.c[j] = (T)pr->patch_weights[j];
  PhaseTimer t0(0, st);
  hipError_t e = launch_prox(a, p.kpw, p.prox_lds, st);
  t0.stop();
  if (e != hipSuccess) return e;

  RowFwdArgs<T> rf;
  rf.g = p.g;
  rf.K = p.K;
  rf.P = p.P;
  rf.rows_per_block = p.rows_per_block;
  rf.acc = a.acc;
  rf.frow = wsp<int>(ws, p.off_frow);
  rf.fcol = wsp<int>(ws, p.off_fcol);
  rf.spec = wsp<C2<T>>(ws, p.off_spec);
  rf.tw = wsp<C2<T>>(ws, p.off_twW);
  rf.plan = p.frow;
  PhaseTimer t1(1, st);
  e = launch_rows_fwd(rf, p.row_ept, p.row_threads, p.row_lds, st);
  t1.stop();
  if (e != hipSuccess) return e;

  double wsum = 0.0;
  for (int j = 0; j < p.L; ++j) {
    const double cj = (double)(T)pr->patch_weights[j];  // the multiplier J applies, rounded to T
    wsum += cj * cj;
  }
  ColArgs<T> ca;
  ca.H = p.H; ca.W = p.W; ca.P = p.P;
  ca.cols_per_block = p.cols_per_block;
  ca.spec = rf.spec;
  ca.tw = wsp<C2<T>>(ws, p.off_twH);
  ca.sx = wsp<double>(ws, p.off_sx);
  ca.sy = wsp<double>(ws, p.off_sy);
  ca.wsum = wsum;
  ca.scale = 1.0 / ((double)p.H * (double)p.W);
  ca.plan = p.fcol;
  PhaseTimer t2(2, st);
  e = launch_cols(ca, p.col_ept, p.col_threads, p.col_lds, st);
  t2.stop();
  if (e != hipSuccess) return e;

  RowInvArgs<T> ri;
  ri.H = p.H; ri.W = p.W; ri.K = p.K; ri.P = p.P;
  ri.rows_per_block = p.rows_per_block;
  ri.spec = rf.spec;
  ri.z = z;
  ri.tw = rf.tw;
  ri.plan = p.frow;
  PhaseTimer t3(3, st);
  e = launch_rows_inv(ri, p.row_ept, p.row_threads, p.row_lds, st);
  t3.stop();
  return e;
}

template <typename T>
segsalsa_status solve_t(const Plan& p, const segsalsa_problem* pr, const void* input, void* z_out, void* ws,
                        segsalsa_stats* stats, hipStream_t st) {
  T* z = reinterpret_cast<T*>(z_out);
  hipError_t e;
  SetupArgs<T> sa;
  sa.g = p.g;
  sa.frow = wsp<int>(ws, p.off_frow);
  sa.fcol = wsp<int>(ws, p.off_fcol);
  sa.H = p.H; sa.W = p.W;
  sa.twW = wsp<C2<T>>(ws, p.off_twW);
  sa.twH = wsp<C2<T>>(ws, p.off_twH);
  sa.sx = wsp<double>(ws, p.off_sx);
  sa.sy = wsp<double>(ws, p.off_sy);
  if ((e = launch_setup(sa, st)) != hipSuccess) return hip_fail(e, "setup kernel");
  if (!pr->warm_start) {
    if ((e = launch_fill_zero(wsp<char>(ws, p.off_flags), 64, st)) != hipSuccess) return hip_fail(e, "fill");
    if ((e = launch_fill_zero(wsp<char>(ws, p.off_d2), p.off_acc - p.off_d2, st)) != hipSuccess)
      return hip_fail(e, "fill");
    InitArgs<T> ia;
    ia.g = p.g;
    ia.K = p.K;
    ia.is_logits = pr->input_is_logits;
    ia.input = reinterpret_cast<const T*>(input);
    ia.z = z;
    ia.phat = wsp<T>(ws, p.off_phat);
    ia.dm = wsp<T>(ws, p.off_dm);
    ia.flags = wsp<int>(ws, p.off_flags);
    if ((e = launch_init(ia, st)) != hipSuccess) return hip_fail(e, "init kernel");
  }
  DiagArgs<T> da;
  std::memset(&da, 0, sizeof(da));
  da.g = p.g;
  da.K = p.K;
  da.pkind = pr->schatten_p == 1.0 ? kSchatten1 : (pr->schatten_p == 2.0 ? kSchatten2 : kSchattenInf);
  da.lambda = pr->lambda;
  for (int j = 0; j < p.L; ++j) {
    da.cw[j] = (double)(T)pr->patch_weights[j];
    da.wsum += da.cw[j] * da.cw[j];
  }
  da.z = z;
  da.zprev = wsp<T>(ws, p.off_zprev);
  da.phat = wsp<T>(ws, p.off_phat);
  da.partial = wsp<double>(ws, p.off_partial);
  da.out = wsp<double>(ws, p.off_out);
  const size_t nel = (size_t)p.K * p.H * p.W;
  const int every = pr->residual_every;
  double rp = 0.0, rd = 0.0;
  int done = 0;
  for (int it = 0; it < pr->iters; ++it) {
    const bool checked = every > 0 && ((it + 1) % every == 0 || it + 1 == pr->iters);
    if (checked && (e = launch_copy(z, da.zprev, nel, st)) != hipSuccess) return hip_fail(e, "copy z");
    if ((e = enqueue_round<T>(p, pr, z, ws, st, checked)) != hipSuccess) return hip_fail(e, "round");
    done = it + 1;
    if (!checked) continue;
    if ((e = launch_reduce(wsp<double>(ws, p.off_restile), p.g.ntiles(), da.out, 0, st)) != hipSuccess)
      return hip_fail(e, "residual reduce");
    if ((e = launch_dual_res(da, st)) != hipSuccess) return hip_fail(e, "dual residual");
    double host[2];
    if ((e = hipMemcpyAsync(host, da.out, sizeof(host), hipMemcpyDeviceToHost, st)) != hipSuccess)
      return hip_fail(e, "residual copy");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "stream sync");
    rp = std::sqrt(std::max(host[0], 0.0));
    rd = pr->mu * std::sqrt(std::max(host[1], 0.0));
    if (pr->tol > 0.0 && rp <= pr->tol && rd <= pr->tol) break;  // stopping rule of Sec. 4
  }
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    int flags = 0;
    double obj = 0.0;
    if (every > 0) {
      if ((e = launch_objective(da, st)) != hipSuccess) return hip_fail(e, "objective");
      if ((e = hipMemcpyAsync(&obj, da.out + 2, sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess)
        return hip_fail(e, "objective copy");
    }
    if ((e = hipMemcpyAsync(&flags, wsp<int>(ws, p.off_flags), sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess)
      return hip_fail(e, "flags copy");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "stream sync");
    stats->flags = flags;
    stats->rounds_done = done;
    stats->primal_res = rp;
    stats->dual_res = rd;
    stats->objective = obj;
  }
  return SEGSALSA_OK;
}

segsalsa_status state_common(const segsalsa_problem* prob, segsalsa_precision precision, const void* ws,
                                    size_t bytes, Plan& p) {
  segsalsa_status s = make_plan(prob, precision, p);
  if (s != SEGSALSA_OK) return s;
  return check_ws(p, ws, bytes);
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
  Plan p;
  segsalsa_status s = make_plan(prob, precision, p);
  if (s != SEGSALSA_OK) return s;
  *bytes = p.total;
  return SEGSALSA_OK;
}

segsalsa_status segsalsa_str_solve(const segsalsa_problem* prob, segsalsa_precision precision, const void* input,
                                   void* z_out, void* workspace, size_t workspace_bytes, segsalsa_stats* stats,
                                   hipStream_t stream) {
  g_last_error.clear();
  Plan p;
  segsalsa_status s = make_plan(prob, precision, p);
  if (s != SEGSALSA_OK) return s;
  if (!z_out) return fail(SEGSALSA_ERR_INVALID_ARG, "z_out is NULL");
  if (!prob->warm_start && !input) return fail(SEGSALSA_ERR_INVALID_ARG, "input is NULL");
  if (input && input == z_out) return fail(SEGSALSA_ERR_INVALID_ARG, "z_out aliases input");
  if (reinterpret_cast<uintptr_t>(z_out) % p.ts || reinterpret_cast<uintptr_t>(input) % p.ts)
    return fail(SEGSALSA_ERR_INVALID_ARG, "input/z_out not aligned to the element size");
  if ((prob->residual_every > 0 || prob->tol > 0.0) && !stats)
    return fail(SEGSALSA_ERR_INVALID_ARG, "residual_every / tol need a stats pointer");
  if ((s = check_ws(p, workspace, workspace_bytes)) != SEGSALSA_OK) return s;
  return p.fp64 ? solve_t<double>(p, prob, input, z_out, workspace, stats, stream)
                : solve_t<float>(p, prob, input, z_out, workspace, stats, stream);
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
  Plan p;
  segsalsa_status s = state_common(prob, precision, workspace, workspace_bytes, p);
  if (s != SEGSALSA_OK) return s;
  void* ws = const_cast<void*>(workspace);
  hipError_t e = p.fp64 ? run_state<double>(p, ws, 1, nullptr, d1, d2, d3, d4, stream)
                        : run_state<float>(p, ws, 1, nullptr, d1, d2, d3, d4, stream);
  return e == hipSuccess ? SEGSALSA_OK : hip_fail(e, "state export kernel");
}

segsalsa_status segsalsa_str_state_import(const segsalsa_problem* prob, segsalsa_precision precision, void* workspace,
                                          size_t workspace_bytes, const void* p_hat, const void* d1, const void* d2,
                                          const void* d3, const void* d4, hipStream_t stream) {
  g_last_error.clear();
  Plan p;
  segsalsa_status s = state_common(prob, precision, workspace, workspace_bytes, p);
  if (s != SEGSALSA_OK) return s;
  if (!p_hat || !d1 || !d2 || !d3 || !d4) return fail(SEGSALSA_ERR_INVALID_ARG, "state import needs all arrays");
  hipError_t e = p.fp64 ? run_state<double>(p, workspace, 0, p_hat, d1, d2, d3, d4, stream)
                        : run_state<float>(p, workspace, 0, p_hat, d1, d2, d3, d4, stream);
  return e == hipSuccess ? SEGSALSA_OK : hip_fail(e, "state import kernel");
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

}  // extern "C"
