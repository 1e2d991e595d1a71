// Host side of librtsgrid: argument validation, the Kaiser-Bessel table, plan
// workspace management and the extern "C" entry points declared in rtsgrid.h.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <utility>

#include "internal.h"

namespace rts {

static thread_local std::string g_error;

void set_error(const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
}

// Modified Bessel function of the first kind, order 0, from its power series
// sum_k ((x/2)^2)^k / (k!)^2 (all terms positive, so no cancellation).
double bessel_i0(double x) {
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 500; ++k) {
    term *= q / ((double)k * (double)k);
    sum += term;
    if (term < 1e-17 * sum) break;
  }
  return sum;
}

// The matrix-core fused step (mfma_bf16x3.hip).
hipError_t launch_grid_resid_mfma(const Plan &P, const TileArgs &a, hipStream_t s);
// Cadence graphs captured from a plan and not yet destroyed (runtime.cpp).
int live_graphs(const Plan *p);

namespace {

#define RTS_HIP(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) {                                                             \
      set_error("%s failed: %s", #expr, hipGetErrorString(e_));                         \
      return e_ == hipErrorOutOfMemory ? RTS_E_NOMEM : RTS_E_HIP;                       \
    }                                                                                   \
  } while (0)

#define RTS_REQUIRE(cond, ...)   \
  do {                           \
    if (!(cond)) {               \
      set_error(__VA_ARGS__);    \
      return RTS_E_INVALID;      \
    }                            \
  } while (0)


// Kaiser-Bessel window of support W, zero at and beyond |t| = W/2.
double kaiser_bessel(double t, int W, double beta) {
  if (!(std::fabs(t) < 0.5 * W)) return 0.0;
  const double a = 2.0 * t / W;
  return bessel_i0(beta * std::sqrt(1.0 - a * a)) / bessel_i0(beta);
}

bool aligned(const void *p, size_t n) { return ((uintptr_t)p % n) == 0; }

// IEEE binary32 -> bfloat16 bits, round to nearest even (finite inputs).
uint16_t bf16_bits(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

float bf16_value(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// Plans whose rts_grid / rts_degrid (and fused step) run the matrix-core kernels.
bool mfma_precision(int p) { return p == RTS_PREC_BF16X3 || p == RTS_PREC_FP32_MFMA; }

rts_status validate(const rts_params *p) {
  RTS_REQUIRE(p != nullptr, "params is NULL");
  RTS_REQUIRE(p->n_grid >= 16 && p->n_grid <= kMaxN && p->n_grid % 2 == 0,
              "n_grid must be even and in [16, %d] (got %d)", kMaxN, p->n_grid);
  const int wmax = mfma_precision(p->precision) ? kMaxWMfma : kMaxW;
  RTS_REQUIRE(p->support >= 2 && p->support <= wmax, "support must be in [2, %d] for this precision (got %d)",
              wmax, p->support);
  RTS_REQUIRE(p->oversample >= 1 && p->oversample <= kMaxOS, "oversample must be in [1, %d] (got %d)",
              kMaxOS, p->oversample);
  RTS_REQUIRE(p->n_chan >= 1 && p->n_base >= 1 && p->n_time >= 1,
              "n_chan, n_base and n_time must be >= 1");
  RTS_REQUIRE(std::isfinite(p->cell_lambda) && p->cell_lambda > 0.0, "cell_lambda must be > 0");
  RTS_REQUIRE(std::isfinite(p->beta), "beta must be finite");
  RTS_REQUIRE(p->conjugate == 0 || p->conjugate == 1, "conjugate must be 0 or 1");
  RTS_REQUIRE(p->precision == RTS_PREC_FP32 || mfma_precision(p->precision), "precision %d is not available",
              p->precision);
  RTS_REQUIRE(p->schedule >= RTS_SCHEDULE_AUTO && p->schedule <= RTS_SCHEDULE_PERSISTENT,
              "schedule %d is not available", p->schedule);
  const int64_t n = (int64_t)p->n_chan * p->n_base * p->n_time * (1 + p->conjugate);
  RTS_REQUIRE(n < ((int64_t)1 << 31), "n_chan*n_base*n_time*(1+conjugate) must be < 2^31");
  // the kernels address one channel's samples with 32-bit byte offsets
  RTS_REQUIRE((int64_t)p->n_base * p->n_time < ((int64_t)1 << 29), "n_base*n_time must be < 2^29");
  RTS_REQUIRE(p->n_grid >= p->support + 2, "n_grid must be at least support + 2");
  if (mfma_precision(p->precision)) {
    RTS_REQUIRE(p->n_grid % 16 == 0, "matrix-core plans need n_grid divisible by 16");
    RTS_REQUIRE(p->tile == 0 || p->tile % 16 == 0, "matrix-core plans need a tile that is a multiple of 16 (got %d)",
                p->tile);
  }
  if (p->tile != 0) {
    RTS_REQUIRE(p->tile >= p->support + 1 && p->tile <= kMaxTile && p->tile % 2 == 0 &&
                    p->n_grid % p->tile == 0,
                "tile must be even, divide n_grid, and lie in [support+1, %d] (got %d)", kMaxTile,
                p->tile);
  }
  return RTS_OK;
}

int choose_tile(int N, int WN) {
  // 64 balances window duplication across tile edges ((64+W)^2/64^2) against LDS
  // per workgroup (64 KiB of complex FP64); fall back to the nearest legal size.
  const int prefs[] = {64, 32, 16};
  for (int t : prefs)
    if (t >= WN && N % t == 0) return t;
  for (int t = kMaxTile; t >= WN; t -= 2)
    if (N % t == 0) return t;
  return 0;
}

int choose_seg_max(int W, int T) {
  if (W <= 8) return T <= 4 ? 4 : 8;
  if (W <= 12) return 4;
  return 2;
}

// Kernel tables of a plan's geometry into caller storage: tab [OS][W], the
// extended table tabE [2*OS][WNP] (zeroed first) and, when hi and lo are given,
// the BF16 hi / lo split of tabE for the matrix-core path.
void fill_tables_raw(const Plan &P, float *tab, float *tabE, uint16_t *hi, uint16_t *lo) {
  const int W = P.W, OS = P.OS;
  for (int p = 0; p < OS; ++p)
    for (int j = 0; j < W; ++j) {
      const int r = P.r0 + p, t = j - P.h_lo;
      tab[(size_t)p * W + j] = (float)kaiser_bessel((double)t - (double)r / OS, W, P.beta);
    }
  // Extended table over the (W+1)-wide window: row s = d*OS + p holds the weights
  // of window columns 0..W for a sample whose cell is d in {0,1} past the window's
  // first tap position, with phase row p.
  for (size_t i = 0; i < (size_t)2 * OS * P.WNP; ++i) {
    tabE[i] = 0.0f;
    if (hi && lo) hi[i] = lo[i] = 0;
  }
  for (int d = 0; d < 2; ++d)
    for (int p = 0; p < OS; ++p)
      for (int i = 0; i < P.WN; ++i) {
        const int j = i - d;
        if (j >= 0 && j < W) {
          const size_t e = (size_t)(d * OS + p) * P.WNP + i;
          tabE[e] = tab[(size_t)p * W + j];
          if (hi && lo) {
            // BF16 hi + lo split of the FP64 kernel value, for the matrix-core path
            const double k = kaiser_bessel((double)(j - P.h_lo) - (double)(P.r0 + p) / OS, W, P.beta);
            hi[e] = bf16_bits((float)k);
            lo[e] = bf16_bits((float)(k - (double)bf16_value(hi[e])));
          }
        }
      }
}

void fill_tables(Plan &P) {
  P.tab.assign((size_t)P.OS * P.W, 0.0f);
  P.tabE.assign((size_t)2 * P.OS * P.WNP, 0.0f);
  P.tab_hi.assign(P.tabE.size(), 0);
  P.tab_lo.assign(P.tabE.size(), 0);
  fill_tables_raw(P, P.tab.data(), P.tabE.data(), P.tab_hi.data(), P.tab_lo.data());
}

// Plan fields that follow from the parameters alone (no allocation): geometry,
// tile edge and samples per segment.
rts_status init_geometry(Plan &P, const rts_params *params) {
  P.p = *params;
  P.N = params->n_grid; P.W = params->support; P.OS = params->oversample;
  P.WN = P.W + 1;
  P.WNP = (P.WN + 3) & ~3;
  P.C = params->n_chan; P.B = params->n_base; P.T = params->n_time;
  P.ncopy = 1 + params->conjugate;
  P.r0 = (P.W & 1) ? -(P.OS / 2) : 0;
  P.h_lo = (P.W & 1) ? (P.W - 1) / 2 : P.W / 2 - 1;
  P.beta = params->beta > 0.0 ? params->beta : 2.34 * P.W;
  P.precision = params->precision;
  P.tile = params->tile ? params->tile : choose_tile(P.N, P.WN);   // 64, 32 or 16
  if (P.tile == 0 || (mfma_precision(P.precision) && P.tile % 16 != 0)) {
    set_error("no legal tile size for n_grid=%d support=%d", P.N, P.W);
    return RTS_E_UNSUPPORTED;
  }
  P.nT = P.N / P.tile;
  P.nT2 = P.nT * P.nT;
  P.nkeys = (int64_t)P.C * P.nT2;
  RTS_REQUIRE(P.nkeys < ((int64_t)1 << 31), "too many (channel, tile) pairs");
  P.seg_max = choose_seg_max(P.W, P.T);
  // supports beyond the FP32 tile kernels' range run on the matrix-core path only
  if (P.W <= kMaxW && !tile_supported(P.W, P.seg_max)) {
    set_error("support %d is not instantiated", P.W);
    return RTS_E_UNSUPPORTED;
  }
  if (mfma_precision(P.precision) && mfma_lds_bytes(P.WN, 2 * P.OS, P.tile) > 65536) {
    set_error("support %d, oversample %d and tile %d need more than 64 KiB of LDS on the matrix-core path",
              P.W, P.OS, P.tile);
    return RTS_E_UNSUPPORTED;
  }
  return RTS_OK;
}

void free_plan(Plan *P) {
  if (!P) return;
  destroy_imager(P);
  hipFree(P->d_tabE);
  hipFree(P->d_tab_hi);
  hipFree(P->d_tab_lo);
  hipFree(P->d_pb_thl);
  hipFree(P->d_pb_tab);
  hipFree(P->d_scale);
  hipFree(P->d_coords);
  hipFree(P->d_list);
  hipFree(P->d_tile_off);
  hipFree(P->d_cursor);
  hipFree(P->d_scan_tmp);
  hipFree(P->d_hist);
  hipFree(P->d_desc);
  hipFree(P->d_order);
  hipFree(P->d_lpt);
  hipFree(P->d_stats);
  hipFree(P->d_chi2_part);
  delete P;
}

// Channels per workgroup of the chunked sort: its LDS histogram holds cg * nT2
// counters (at most 8192, 32 KiB).
int chunk_channels(int nT2) { return std::max(1, std::min(kMaxCg, 8192 / nT2)); }

// Choose the chunked counting sort when the tracks are short enough for the lane
// path and one channel's tiles fit the LDS histogram; the (key, chunk) count
// matrix is kept near 4M entries (max_hist entries at most).
void choose_sort(Plan &P, int64_t max_hist = (int64_t)8 << 20) {
  P.nbx = 0;
  P.chunk = 0;
  P.cg = 1;
  if (P.T > 64 || P.nT2 > 8192) return;
  int g = 1;
  while (g < P.T) g <<= 1;
  const int64_t per_iter = kBlock / g;
  const int64_t ntr = (int64_t)P.ncopy * P.B;
  const int64_t max_nbx = std::max<int64_t>(1, (ntr + per_iter - 1) / per_iter);
  const int64_t cap_nbx = std::max<int64_t>(1, max_hist / P.nkeys);
  // The most channels per workgroup (uvw reuse) that still gives >= 1024 workgroups.
  int64_t nbx = 1;
  for (int cg = chunk_channels(P.nT2); cg >= 1; cg /= 2) {
    const int64_t groups = (P.C + cg - 1) / cg;
    nbx = std::min(max_nbx, cap_nbx);
    P.cg = cg;
    if (groups * nbx >= 1024) break;
  }
  nbx = std::max<int64_t>(nbx, 1);
  int64_t chunk = (ntr + nbx - 1) / nbx;
  chunk = (chunk + per_iter - 1) / per_iter * per_iter;
  nbx = (ntr + chunk - 1) / chunk;
  P.nbx = (int)nbx;
  P.chunk = chunk;
}

PlanArgs plan_args(const Plan &P, const double *uvw, const float *w) {
  PlanArgs a{};
  a.uvw = uvw;
  a.scale = P.d_scale;
  a.w = w;
  a.coords = P.d_coords;
  a.list = P.d_list;
  a.counts = P.d_cursor;
  a.stats = P.d_stats;
  a.list_cap = P.list_cap;
  a.N = P.N; a.W = P.W; a.OS = P.OS; a.WN = P.WN; a.r0 = P.r0; a.h_lo = P.h_lo;
  a.log2os = -1;
  for (int l = 0; l <= 6; ++l)
    if ((1 << l) == P.OS) a.log2os = l;
  a.log2tile = -1;
  for (int l = 1; l <= 13; ++l)
    if ((1 << l) == P.tile) a.log2tile = l;
  a.tile = P.tile; a.nT = P.nT; a.nT2 = P.nT2;
  a.C = P.C; a.B = P.B; a.T = P.T; a.ncopy = P.ncopy; a.seg_max = P.seg_max;
  // Tracks of up to 64 samples: one lane per sample, channels in groups of 8 so
  // that each lane's uvw is loaded once per group.
  a.tgroup = 0;
  if (P.T <= 64) {
    int g = 1;
    while (g < P.T) g <<= 1;
    a.tgroup = g;
  }
  // per-track path: LDS histogram over the channels of a workgroup when it fits in 32 KiB
  a.nbx = P.nbx;
  a.chunk = P.chunk;
  a.vec_t = (P.T == 8 || P.T == 4) && aligned(w, 16);
  a.hist = P.d_hist;
  a.offs = P.d_hist;
  a.tile_off = P.d_tile_off;
  a.nkeys = P.nkeys;
  a.desc = P.d_desc;
  if (P.nbx > 0) {
    a.use_lds = 0;
    a.cg = P.cg;
  } else if (a.tgroup > 0) {
    a.use_lds = 0;
    a.cg = 8;
  } else if (P.nT2 <= 8192) {
    a.use_lds = 1;
    a.cg = std::max(1, std::min(8, 8192 / P.nT2));
  } else {
    a.use_lds = 0;
    a.cg = 8;
  }
  return a;
}

// Exclusive scan of the listing counts into tile offsets (and cursors or
// per-chunk offsets for the scatter pass).
hipError_t scan_counts(const Plan &P, hipStream_t s) {
  if (P.nbx > 0) return launch_hist_scan(P.d_hist, P.nbx, P.nkeys, P.d_cursor, P.d_tile_off, P.d_scan_tmp, s);
  return launch_scan(P.d_cursor, P.d_tile_off, P.d_cursor, P.d_scan_tmp, P.nkeys, s);
}

TileArgs tile_args(const Plan &P) {
  TileArgs a{};
  a.list = P.d_list;
  a.tile_off = P.d_tile_off;
  a.coords = P.d_coords;
  a.tabE = P.d_tabE;
  a.chi2_part = P.d_chi2_part;
  a.list_cap = P.list_cap;
  a.N = P.N; a.tile = P.tile; a.nT = P.nT; a.nT2 = P.nT2; a.nkeys = (int)P.nkeys;
  a.B = P.B; a.T = P.T; a.ncopy = P.ncopy;
  a.OS2 = 2 * P.OS; a.WNP = P.WNP; a.WN = P.WN;
  a.vec = 0;
  a.seg_max = P.seg_max;
  a.order = P.d_order;
  a.queue = P.d_lpt ? P.d_lpt + kLptQueue : nullptr;
  return a;
}

template <class T>
hipError_t dalloc(T **p, size_t n) {
  return hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T));
}

// Whole-track segments can use vector loads/stores when every track is exactly
// one segment's length and the per-sample arrays are 16-byte aligned.
int vector_ok(const Plan &P, const void *vis, const void *w, const void *model) {
  if (P.T != P.seg_max || (P.seg_max != 4 && P.seg_max != 8)) return 0;
  if ((vis && !aligned(vis, 16)) || (w && !aligned(w, 16)) || (model && !aligned(model, 16))) return 0;
  return 1;
}

rts_status check_plan(rts_plan_t plan) {
  RTS_REQUIRE(plan != nullptr, "plan is NULL");
  return RTS_OK;
}

}  // namespace

bool tile_supported(int W, int seg_max) {
  if (W < 2 || W > kMaxW) return false;
  if (W <= 8) return seg_max == 4 || seg_max == 8;
  if (W <= 12) return seg_max == 4;
  return seg_max == 2;
}

hipError_t launch_tile(int mode, const Plan &P, const TileArgs &a, hipStream_t s) {
  switch (mode) {
    case kGrid: return launch_tile_mode<kGrid>(P, a, s, false);
    case kDegrid: return launch_tile_mode<kDegrid>(P, a, s, false);
    default: return launch_tile_mode<kFused>(P, a, s, false);
  }
}

// ------------------------------------------------ allocation-free fused step
// Workspace of rts_grid_degrid_noalloc: one static array per device, held from
// the library's load until the process ends.  Host code never uses the array's
// name as an address: its device address is looked up once per device with
// hipGetSymbolAddress and kept in g_scratch_addr.
constexpr size_t kScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices];

// Device address of the current device's scratch array (looked up on the first
// call on each device, with that device current).
hipError_t scratch_addr(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return hipSuccess;
}

// Small host values reach the device as kernel arguments (no host buffer has to
// outlive the call and no copy engine is involved): 240 words per launch.
constexpr int kWordsPerStore = 240;
struct StoreWords {
  uint32_t w[kWordsPerStore];
};

__global__ __launch_bounds__(256) void k_store_words(uint32_t *dst, StoreWords v, int n) {
  if ((int)threadIdx.x < n) dst[threadIdx.x] = v.w[threadIdx.x];
}

hipError_t store_words(void *dst, const void *src, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 4;
  const unsigned char *b = (const unsigned char *)src;
  for (size_t i = 0; i < n; i += kWordsPerStore) {
    StoreWords v{};
    const int m = (int)std::min<size_t>(kWordsPerStore, n - i);
    std::memcpy(v.w, b + 4 * i, 4 * (size_t)m);
    hipLaunchKernelGGL(k_store_words, dim3(1), dim3(256), 0, s, (uint32_t *)dst + i, v, m);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Bump allocator over the scratch array (256-byte aligned regions).
struct Carve {
  unsigned char *base;
  size_t used = 0;
  template <class T>
  T *take(size_t n) {
    used = (used + 255) & ~(size_t)255;
    T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
    used += std::max<size_t>(n, 1) * sizeof(T);
    return p;
  }
};

// Lays the plan workspace out in `base` (nullptr: only measure) and returns the
// bytes it needs.  The work list holds the worst case, four listings per sample
// (every segment has at least one sample and touches at most 2 x 2 tiles), so no
// listing can be dropped.
size_t carve_plan(Plan &P, unsigned char *base, int64_t max_hist) {
  Carve cv{base};
  const int64_t nsamp = (int64_t)P.C * P.B * P.T;
  choose_sort(P, max_hist);
  P.scan_blocks = (P.nkeys + 4095) / 4096;
  P.d_tabE = cv.take<float>((size_t)2 * P.OS * P.WNP);
  P.d_scale = cv.take<double>((size_t)P.C);
  P.d_stats = cv.take<unsigned long long>(8);
  P.d_tile_off = cv.take<uint32_t>((size_t)P.nkeys + 1);
  P.d_cursor = cv.take<uint32_t>((size_t)P.nkeys);
  P.d_scan_tmp = cv.take<uint32_t>((size_t)P.scan_blocks + 1);
  P.d_chi2_part = cv.take<double>((size_t)P.nkeys);
  P.d_coords = cv.take<uint16_t>((size_t)nsamp);
  if (P.nbx > 0) {
    P.d_desc = cv.take<uint32_t>((size_t)P.C * P.B);
    P.d_hist = cv.take<uint32_t>((size_t)P.nbx * P.nkeys);
  }
  P.list_cap = 4 * nsamp;
  P.d_list = cv.take<uint2>((size_t)P.list_cap);
  return cv.used;
}

}  // namespace

hipError_t prepare_tile_kernels(const Plan &P) {
  TileArgs a{};
  a.OS2 = 2 * P.OS;
  a.WNP = P.WNP;
  hipError_t e = launch_tile_mode<kGrid>(P, a, nullptr, true);
  if (e == hipSuccess) e = launch_tile_mode<kDegrid>(P, a, nullptr, true);
  if (e == hipSuccess) e = launch_tile_mode<kFused>(P, a, nullptr, true);
  return e;
}

}  // namespace rts

using namespace rts;


extern "C" {

const char *rts_last_error(void) { return g_error.c_str(); }

const char *rts_version(void) { return "rtsgrid 0.1 (gfx950)"; }

rts_status rts_grid_plan(rts_plan_t *out, const rts_params *params, const double *uvw_m,
                         const double *freq_hz, const float *weights, void *stream) {
  RTS_REQUIRE(out != nullptr, "out is NULL");
  *out = nullptr;
  if (rts_status st = validate(params)) return st;
  RTS_REQUIRE(uvw_m && freq_hz && weights, "uvw_m, freq_hz and weights must be non-NULL");
  RTS_REQUIRE(aligned(uvw_m, 8) && aligned(weights, 4), "uvw_m / weights are misaligned");
  for (int c = 0; c < params->n_chan; ++c)
    RTS_REQUIRE(std::isfinite(freq_hz[c]) && freq_hz[c] > 0.0, "freq_hz[%d] must be > 0", c);

  std::unique_ptr<Plan, void (*)(Plan *)> P(new (std::nothrow) Plan(), [](Plan *p) { free_plan(p); });
  if (!P) {
    set_error("host allocation failed");
    return RTS_E_NOMEM;
  }
  if (rts_status st = init_geometry(*P, params)) return st;
  fill_tables(*P);
  RTS_HIP(hipGetDevice(&P->device));
  RTS_HIP(hipDeviceGetAttribute(&P->n_cu, hipDeviceAttributeMultiprocessorCount, P->device));
  P->schedule = params->schedule == RTS_SCHEDULE_AUTO ? RTS_SCHEDULE_TILES : params->schedule;
  if (P->W <= kMaxW) RTS_HIP(prepare_tile_kernels(*P));
  hipStream_t s = (hipStream_t)stream;

  const int64_t nsamp = (int64_t)P->C * P->B * P->T;
  choose_sort(*P);
  const int64_t nhist = P->nbx > 0 ? P->nkeys * P->nbx : 0;
  P->scan_blocks = (P->nkeys + 4095) / 4096;
  RTS_HIP(dalloc(&P->d_tabE, P->tabE.size()));
  RTS_HIP(dalloc(&P->d_tab_hi, P->tab_hi.size()));
  RTS_HIP(dalloc(&P->d_tab_lo, P->tab_lo.size()));
  RTS_HIP(dalloc(&P->d_scale, (size_t)P->C));
  RTS_HIP(dalloc(&P->d_coords, (size_t)nsamp * P->ncopy));
  RTS_HIP(dalloc(&P->d_tile_off, (size_t)P->nkeys + 1));
  RTS_HIP(dalloc(&P->d_cursor, (size_t)P->nkeys));
  RTS_HIP(dalloc(&P->d_scan_tmp, (size_t)P->scan_blocks + 1));
  RTS_HIP(dalloc(&P->d_stats, 8));
  RTS_HIP(dalloc(&P->d_chi2_part, (size_t)P->nkeys));
  if (P->nbx > 0) {
    RTS_HIP(dalloc(&P->d_hist, (size_t)nhist));
    RTS_HIP(dalloc(&P->d_desc, (size_t)P->C * P->ncopy * P->B));
  }
  // Longest-first order: for the persistent launch, and for the matrix-core
  // kernels when there are few tiles per resident workgroup (at most 64 per CU,
  // about 20 per workgroup slot), where a few dense tiles otherwise run last;
  // with more tiles the tail is short and the ordering pass costs more than it
  // saves.
  const bool mfma_order = mfma_precision(P->precision) && P->nkeys <= (int64_t)64 * P->n_cu;
  if (P->schedule == RTS_SCHEDULE_PERSISTENT || mfma_order) {
    RTS_HIP(dalloc(&P->d_order, (size_t)P->nkeys));
    RTS_HIP(dalloc(&P->d_lpt, (size_t)kLptWords));
  }

  std::vector<double> scale(P->C);
  for (int c = 0; c < P->C; ++c) scale[c] = freq_hz[c] / (kCLight * params->cell_lambda);
  RTS_HIP(hipMemcpyAsync(P->d_tabE, P->tabE.data(), P->tabE.size() * sizeof(float),
                         hipMemcpyHostToDevice, s));
  RTS_HIP(hipMemcpyAsync(P->d_scale, scale.data(), scale.size() * sizeof(double),
                         hipMemcpyHostToDevice, s));
  RTS_HIP(hipMemcpyAsync(P->d_tab_hi, P->tab_hi.data(), P->tab_hi.size() * 2, hipMemcpyHostToDevice, s));
  RTS_HIP(hipMemcpyAsync(P->d_tab_lo, P->tab_lo.data(), P->tab_lo.size() * 2, hipMemcpyHostToDevice, s));
  RTS_HIP(launch_fill_u32(P->d_cursor, P->nkeys, 0u, s));
  RTS_HIP(launch_fill_u32((uint32_t *)P->d_stats, 16, 0u, s));

  PlanArgs pa = plan_args(*P, uvw_m, weights);
  RTS_HIP(launch_plan_count(pa, s));
  RTS_HIP(scan_counts(*P, s));
  unsigned long long stats[8] = {0};
  uint32_t total = 0;
  RTS_HIP(hipMemcpyAsync(stats, P->d_stats, sizeof stats, hipMemcpyDeviceToHost, s));
  RTS_HIP(hipMemcpyAsync(&total, P->d_tile_off + P->nkeys, sizeof total, hipMemcpyDeviceToHost, s));
  RTS_HIP(hipStreamSynchronize(s));
  if ((int64_t)stats[4] != (int64_t)total) {
    set_error("work-list count mismatch (%llu listed, %u scanned)", stats[4], total);
    return RTS_E_HIP;
  }
  // headroom for later rts_plan_update calls whose flags or uv coverage differ
  P->list_cap = std::max<int64_t>((int64_t)total + (int64_t)total / 8 + 1024, 1);
  P->list_cap = std::min<int64_t>(P->list_cap, (int64_t)UINT32_MAX);
  RTS_HIP(dalloc(&P->d_list, (size_t)P->list_cap));
  pa.list = P->d_list;
  pa.list_cap = P->list_cap;
  RTS_HIP(launch_plan_scatter(pa, s));
  if (P->d_order) RTS_HIP(launch_lpt_order(P->d_tile_off, P->nkeys, P->d_lpt, P->d_order, s));

  rts_plan_info &I = P->info;
  I.n_samples = nsamp;
  I.n_valid = (int64_t)stats[0];
  I.n_flagged = (int64_t)stats[1];
  I.n_offgrid = (int64_t)stats[2];
  I.n_segments = (int64_t)stats[3];
  I.n_listings = (int64_t)total;
  I.n_dropped = 0;
  I.tile = P->tile;
  I.seg_max = P->seg_max;
  I.workspace_bytes = (int64_t)(P->tabE.size() * 4 + P->C * 8 + nsamp * P->ncopy * 2 +
                                (P->nkeys + 1) * 4 + P->nkeys * 4 + (P->scan_blocks + 1) * 4 + 64 +
                                (P->nbx > 0 ? nhist * 4 + (int64_t)P->C * P->ncopy * P->B * 4 : 0) +
                                P->nkeys * 8 + P->list_cap * 8 +
                                (P->d_order ? P->nkeys * 4 + kLptWords * 4 : 0));
  *out = P.release();
  return RTS_OK;
}

rts_status rts_plan_update(rts_plan_t plan, const double *uvw_m, const float *weights, void *stream) {
  if (rts_status st = check_plan(plan)) return st;
  RTS_REQUIRE(uvw_m && weights, "uvw_m and weights must be non-NULL");
  RTS_REQUIRE(aligned(uvw_m, 8) && aligned(weights, 4), "uvw_m / weights are misaligned");
  hipStream_t s = (hipStream_t)stream;
  PlanArgs pa = plan_args(*plan, uvw_m, weights);
  RTS_HIP(launch_fill_u32(plan->d_cursor, plan->nkeys, 0u, s));
  RTS_HIP(launch_fill_u32((uint32_t *)plan->d_stats, 16, 0u, s));
  RTS_HIP(launch_plan_count(pa, s));
  RTS_HIP(scan_counts(*plan, s));
  RTS_HIP(launch_plan_scatter(pa, s));
  if (plan->d_order) RTS_HIP(launch_lpt_order(plan->d_tile_off, plan->nkeys, plan->d_lpt, plan->d_order, s));
  plan->stats_pending = true;
  return RTS_OK;
}

rts_status rts_grid(rts_plan_t plan, const float *vis, const float *weights, float *grid,
                    void *stream) {
  if (rts_status st = check_plan(plan)) return st;
  RTS_REQUIRE(vis && weights && grid, "vis, weights and grid must be non-NULL");
  RTS_REQUIRE(aligned(vis, 8) && aligned(weights, 4) && aligned(grid, 16),
              "vis must be 8-byte, weights 4-byte and grid 16-byte aligned");
  TileArgs a = tile_args(*plan);
  a.vis = (const float2 *)vis;
  a.w = weights;
  a.gout = (float2 *)grid;
  a.vec = vector_ok(*plan, vis, weights, nullptr);
  if (mfma_precision(plan->precision))
    RTS_HIP(launch_grid_mfma(*plan, a, (hipStream_t)stream));
  else
    RTS_HIP(launch_tile(kGrid, *plan, a, (hipStream_t)stream));
  return RTS_OK;
}

rts_status rts_degrid(rts_plan_t plan, const float *grid, float *vis_out, void *stream) {
  if (rts_status st = check_plan(plan)) return st;
  RTS_REQUIRE(grid && vis_out, "grid and vis_out must be non-NULL");
  RTS_REQUIRE(aligned(grid, 8) && aligned(vis_out, 8), "grid and vis_out must be 8-byte aligned");
  TileArgs a = tile_args(*plan);
  a.gin = (const float2 *)grid;
  a.model = (float2 *)vis_out;
  a.vec = vector_ok(*plan, nullptr, nullptr, vis_out);
  if (mfma_precision(plan->precision))
    RTS_HIP(launch_degrid_mfma(*plan, a, (hipStream_t)stream));
  else
    RTS_HIP(launch_tile(kDegrid, *plan, a, (hipStream_t)stream));
  return RTS_OK;
}

rts_status rts_grid_degrid(rts_plan_t plan, const float *vis, const float *weights,
                           const float *grid_in, float *model_out, float *grid_out,
                           double *chi2_out, void *stream) {
  if (rts_status st = check_plan(plan)) return st;
  if (plan->ncopy != 1) {
    set_error("rts_grid_degrid does not support plans built with conjugate=1");
    return RTS_E_UNSUPPORTED;
  }
  if (!mfma_precision(plan->precision) && (plan->W > kMaxW || plan->d_pb_thl)) {
    set_error("the fused step of an FP32 plan needs support <= %d and the shared kernel", kMaxW);
    return RTS_E_UNSUPPORTED;
  }
  RTS_REQUIRE(vis && weights && grid_in && grid_out, "vis, weights, grid_in, grid_out must be non-NULL");
  RTS_REQUIRE(aligned(vis, 8) && aligned(weights, 4) && aligned(grid_in, 8) && aligned(grid_out, 16) &&
                  aligned(model_out, 8) && aligned(chi2_out, 8),
              "misaligned buffer");
  const size_t gbytes = (size_t)plan->C * plan->N * plan->N * 8;
  const char *gi = (const char *)grid_in, *go = (const char *)grid_out;
  RTS_REQUIRE(gi + gbytes <= go || go + gbytes <= gi, "grid_in and grid_out overlap");
  if (model_out) {
    // the model is written while the visibilities, weights and G_in are still read
    const size_t n = (size_t)plan->C * plan->B * plan->T;
    const char *m = (const char *)model_out;
    auto apart = [&](const void *p, size_t bytes) {
      const char *q = (const char *)p;
      return m + 8 * n <= q || q + bytes <= m;
    };
    RTS_REQUIRE(apart(vis, 8 * n) && apart(weights, 4 * n) && apart(grid_in, gbytes) && apart(grid_out, gbytes),
                "model_out overlaps vis, weights, grid_in or grid_out");
  }
  TileArgs a = tile_args(*plan);
  a.vis = (const float2 *)vis;
  a.w = weights;
  a.gin = (const float2 *)grid_in;
  a.gout = (float2 *)grid_out;
  a.model = (float2 *)model_out;
  a.write_model = model_out != nullptr;
  a.vec = vector_ok(*plan, vis, weights, model_out);
  hipStream_t s = (hipStream_t)stream;
  if (mfma_precision(plan->precision)) {
    // matrix-core plans: degrid into model_out, then grid w (V - M), which also
    // leaves the chi2 partial sums per key
    RTS_REQUIRE(model_out != nullptr, "the fused step of a matrix-core plan needs model_out");
    RTS_HIP(launch_degrid_mfma(*plan, a, s));
    RTS_HIP(launch_grid_resid_mfma(*plan, a, s));
    if (chi2_out) RTS_HIP(launch_chi2_reduce(plan->d_chi2_part, plan->nkeys, chi2_out, s));
    return RTS_OK;
  }
  RTS_HIP(launch_tile(kFused, *plan, a, s));
  if (chi2_out) RTS_HIP(launch_chi2_reduce(plan->d_chi2_part, plan->nkeys, chi2_out, s));
  return RTS_OK;
}

rts_status rts_grid_degrid_noalloc(const rts_params *params, const double *uvw_m, const double *freq_hz,
                                   const float *weights, const float *vis, const float *grid_in, float *model_out,
                                   float *grid_out, double *chi2_out, void *stream) {
  if (rts_status st = validate(params)) return st;
  RTS_REQUIRE(params->precision == RTS_PREC_FP32, "rts_grid_degrid_noalloc supports FP32 plans only");
  if (params->conjugate) {
    set_error("rts_grid_degrid_noalloc does not support conjugate=1 (as rts_grid_degrid)");
    return RTS_E_UNSUPPORTED;
  }
  RTS_REQUIRE(uvw_m && freq_hz && weights && vis && grid_in && grid_out,
              "uvw_m, freq_hz, weights, vis, grid_in and grid_out must be non-NULL");
  RTS_REQUIRE(aligned(uvw_m, 8) && aligned(weights, 4) && aligned(vis, 8) && aligned(grid_in, 8) &&
                  aligned(grid_out, 16) && aligned(model_out, 8) && aligned(chi2_out, 8),
              "misaligned buffer");
  for (int c = 0; c < params->n_chan; ++c)
    RTS_REQUIRE(std::isfinite(freq_hz[c]) && freq_hz[c] > 0.0, "freq_hz[%d] must be > 0", c);
  Plan P;   // host-side description only: its device arrays are carved from the scratch array
  if (rts_status st = init_geometry(P, params)) return st;
  RTS_REQUIRE(P.W <= kMaxW, "rts_grid_degrid_noalloc supports support <= %d", kMaxW);
  P.schedule = RTS_SCHEDULE_TILES;
  const size_t n = (size_t)P.C * P.B * P.T;
  const size_t gbytes = (size_t)P.C * P.N * P.N * 8;
  const char *gi = (const char *)grid_in, *go = (const char *)grid_out;
  RTS_REQUIRE(gi + gbytes <= go || go + gbytes <= gi, "grid_in and grid_out overlap");
  if (model_out) {
    const char *m = (const char *)model_out;
    auto apart = [&](const void *p, size_t bytes) {
      const char *q = (const char *)p;
      return m + 8 * n <= q || q + bytes <= m;
    };
    RTS_REQUIRE(apart(vis, 8 * n) && apart(weights, 4 * n) && apart(grid_in, gbytes) && apart(grid_out, gbytes),
                "model_out overlaps vis, weights, grid_in or grid_out");
  }
  // Size check before any device work: everything but the chunked sort's count
  // matrix must fit; the matrix then takes at most a quarter of what is left.
  int64_t max_hist = 1;
  {
    Plan Q = P;
    const size_t with_one = carve_plan(Q, nullptr, 1);
    const size_t hist_one = Q.nbx > 0 ? (size_t)Q.nbx * Q.nkeys * 4 + 256 : 0;
    const size_t fixed = with_one - hist_one;
    RTS_REQUIRE(fixed <= kScratchBytes,
                "this problem needs %zu bytes of plan workspace; rts_grid_degrid_noalloc has %zu "
                "(use rts_grid_plan + rts_grid_degrid)", fixed, kScratchBytes);
    max_hist = std::max<int64_t>(((int64_t)kScratchBytes - (int64_t)fixed) / 16 - 64, 1);
  }
  int dev = 0;
  RTS_HIP(hipGetDevice(&dev));
  RTS_HIP(hipDeviceGetAttribute(&P.n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  P.device = dev;
  RTS_HIP(prepare_tile_kernels(P));
  void *base = nullptr;
  RTS_HIP(scratch_addr(&base));
  const size_t need = carve_plan(P, (unsigned char *)base, max_hist);
  RTS_REQUIRE(need <= kScratchBytes,
              "this problem needs %zu bytes of plan workspace; rts_grid_degrid_noalloc has %zu "
              "(use rts_grid_plan + rts_grid_degrid)", need, kScratchBytes);
  hipStream_t s = (hipStream_t)stream;
  // kernel table and per-channel scales, as kernel arguments
  {
    float tab[kMaxOS * kMaxW];
    float tabE[2 * kMaxOS * ((kMaxW + 1 + 3) & ~3)];
    fill_tables_raw(P, tab, tabE, nullptr, nullptr);
    RTS_HIP(store_words(P.d_tabE, tabE, (size_t)2 * P.OS * P.WNP * sizeof(float), s));
    double sc[kWordsPerStore / 2];
    for (int c0 = 0; c0 < P.C; c0 += kWordsPerStore / 2) {
      const int m = std::min(P.C - c0, kWordsPerStore / 2);
      for (int i = 0; i < m; ++i) sc[i] = freq_hz[c0 + i] / (kCLight * params->cell_lambda);
      RTS_HIP(store_words(P.d_scale + c0, sc, (size_t)m * sizeof(double), s));
    }
  }
  // plan: coordinates, segments, counting sort (as rts_plan_update)
  PlanArgs pa = plan_args(P, uvw_m, weights);
  RTS_HIP(launch_fill_u32(P.d_cursor, P.nkeys, 0u, s));
  RTS_HIP(launch_fill_u32((uint32_t *)P.d_stats, 16, 0u, s));
  RTS_HIP(launch_plan_count(pa, s));
  RTS_HIP(scan_counts(P, s));
  RTS_HIP(launch_plan_scatter(pa, s));
  // fused residual step (as rts_grid_degrid)
  TileArgs a = tile_args(P);
  a.vis = (const float2 *)vis;
  a.w = weights;
  a.gin = (const float2 *)grid_in;
  a.gout = (float2 *)grid_out;
  a.model = (float2 *)model_out;
  a.write_model = model_out != nullptr;
  a.vec = vector_ok(P, vis, weights, model_out);
  RTS_HIP(launch_tile(kFused, P, a, s));
  if (chi2_out) RTS_HIP(launch_chi2_reduce(P.d_chi2_part, P.nkeys, chi2_out, s));
  return RTS_OK;
}

rts_status rts_grid_backward(rts_plan_t plan, const float *vis, const float *weights, const float *grad_grid,
                             float *grad_vis, float *grad_weights, void *stream) {
  if (rts_status st = check_plan(plan)) return st;
  if (plan->ncopy != 1) {
    set_error("rts_grid_backward does not support plans built with conjugate=1");
    return RTS_E_UNSUPPORTED;
  }
  RTS_REQUIRE(vis && weights && grad_grid && grad_vis, "vis, weights, grad_grid and grad_vis must be non-NULL");
  RTS_REQUIRE(aligned(vis, 8) && aligned(weights, 4) && aligned(grad_grid, 8) && aligned(grad_vis, 8) &&
                  aligned(grad_weights, 4),
              "misaligned buffer");
  const size_t n = (size_t)plan->C * plan->B * plan->T;
  const size_t gbytes = (size_t)plan->C * plan->N * plan->N * 8;
  auto apart = [](const void *p, size_t pb, const void *q, size_t qb) {
    const char *a = (const char *)p, *b = (const char *)q;
    return !a || !b || a + pb <= b || b + qb <= a;
  };
  RTS_REQUIRE(apart(grad_vis, 8 * n, vis, 8 * n) && apart(grad_vis, 8 * n, weights, 4 * n) &&
                  apart(grad_vis, 8 * n, grad_grid, gbytes) && apart(grad_weights, 4 * n, vis, 8 * n) &&
                  apart(grad_weights, 4 * n, weights, 4 * n) && apart(grad_weights, 4 * n, grad_grid, gbytes) &&
                  apart(grad_weights, 4 * n, grad_vis, 8 * n),
              "grad_vis / grad_weights overlap another buffer");
  hipStream_t s = (hipStream_t)stream;
  if (rts_status st = rts_degrid(plan, grad_grid, grad_vis, stream)) return st;
  RTS_HIP(launch_grid_backward((const float2 *)vis, weights, (float2 *)grad_vis, grad_weights, (int64_t)n, s));
  return RTS_OK;
}

rts_status rts_chi2_backward(rts_plan_t plan, const float *vis, const float *weights, const float *model,
                             const float *grid_resid, const double *grad_chi2, float *grad_vis,
                             float *grad_weights, float *grad_grid, void *stream) {
  if (rts_status st = check_plan(plan)) return st;
  if (plan->ncopy != 1) {
    set_error("rts_chi2_backward does not support plans built with conjugate=1");
    return RTS_E_UNSUPPORTED;
  }
  RTS_REQUIRE(grad_chi2 != nullptr, "grad_chi2 must be non-NULL");
  RTS_REQUIRE(!(grad_vis || grad_weights) || (vis && weights && model),
              "vis, weights and model are needed for grad_vis / grad_weights");
  RTS_REQUIRE(!grad_grid || grid_resid, "grid_resid is needed for grad_grid");
  RTS_REQUIRE(aligned(vis, 8) && aligned(weights, 4) && aligned(model, 8) && aligned(grid_resid, 16) &&
                  aligned(grad_chi2, 8) && aligned(grad_vis, 8) && aligned(grad_weights, 4) && aligned(grad_grid, 16),
              "misaligned buffer (grids need 16-byte alignment)");
  const size_t n = (size_t)plan->C * plan->B * plan->T;
  const size_t gbytes = (size_t)plan->C * plan->N * plan->N * 8;
  auto apart = [](const void *p, size_t pb, const void *q, size_t qb) {
    const char *a = (const char *)p, *b = (const char *)q;
    return !a || !b || a + pb <= b || b + qb <= a;
  };
  const std::pair<const void *, size_t> ins[] = {{vis, 8 * n}, {weights, 4 * n}, {model, 8 * n}};
  for (const auto &in : ins) {
    RTS_REQUIRE(apart(grad_vis, 8 * n, in.first, in.second) && apart(grad_weights, 4 * n, in.first, in.second),
                "grad_vis / grad_weights overlap an input");
  }
  RTS_REQUIRE(apart(grad_vis, 8 * n, grad_weights, 4 * n), "grad_vis and grad_weights overlap");
  RTS_REQUIRE(apart(grad_grid, gbytes, vis, 8 * n) && apart(grad_grid, gbytes, model, 8 * n) &&
                  apart(grad_grid, gbytes, weights, 4 * n) && apart(grad_grid, gbytes, grad_vis, 8 * n) &&
                  apart(grad_grid, gbytes, grad_weights, 4 * n) && apart(grad_grid, gbytes, grad_chi2, 8),
              "grad_grid overlaps another buffer");
  RTS_REQUIRE(grad_grid == grid_resid || apart(grad_grid, gbytes, grid_resid, gbytes),
              "grad_grid partly overlaps grid_resid");
  RTS_HIP(launch_chi2_backward(*plan, (const float2 *)vis, weights, (const float2 *)model, grad_chi2,
                               (float2 *)grad_vis, grad_weights, (const float2 *)grid_resid, (float2 *)grad_grid,
                               (hipStream_t)stream));
  return RTS_OK;
}

rts_status rts_compute_coords(const rts_params *params, const double *uvw_m, const double *freq_hz,
                              const float *weights, int32_t *out, void *stream) {
  if (rts_status st = validate(params)) return st;
  RTS_REQUIRE(uvw_m && freq_hz && weights && out, "null pointer argument");
  hipStream_t s = (hipStream_t)stream;
  std::vector<double> scale(params->n_chan);
  for (int c = 0; c < params->n_chan; ++c) scale[c] = freq_hz[c] / (kCLight * params->cell_lambda);
  double *d_scale = nullptr;
  RTS_HIP(dalloc(&d_scale, scale.size()));
  hipError_t e = hipMemcpyAsync(d_scale, scale.data(), scale.size() * sizeof(double),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = launch_coords(uvw_m, d_scale, weights, out, params->n_grid, params->support,
                      params->oversample, params->n_chan, params->n_base, params->n_time, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipFree(d_scale);
  RTS_HIP(e);
  return RTS_OK;
}

rts_status rts_plan_valid_mask(rts_plan_t plan, uint8_t *mask, void *stream) {
  if (rts_status st = check_plan(plan)) return st;
  RTS_REQUIRE(mask != nullptr, "mask is NULL");
  const int64_t n = (int64_t)plan->C * plan->B * plan->T;
  RTS_HIP(launch_valid_mask(plan->d_coords, mask, plan->B, plan->T, plan->ncopy, n, (hipStream_t)stream));
  return RTS_OK;
}

rts_status rts_stream_copy(const void *src, void *dst, int64_t bytes, void *stream) {
  RTS_REQUIRE(bytes >= 0, "bytes must be >= 0");
  if (bytes == 0) return RTS_OK;
  RTS_REQUIRE(src && dst, "src and dst must be non-NULL");
  RTS_REQUIRE(aligned(src, 16) && aligned(dst, 16), "src and dst must be 16-byte aligned");
  const char *a = (const char *)src, *b = (const char *)dst;
  RTS_REQUIRE(a + bytes <= b || b + bytes <= a, "src and dst overlap");
  int dev = 0, n_cu = 256;
  RTS_HIP(hipGetDevice(&dev));
  RTS_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  RTS_HIP(launch_stream_copy(src, dst, bytes, n_cu, (hipStream_t)stream));
  return RTS_OK;
}

rts_status rts_plan_set_baseline_kernels(rts_plan_t plan, const float *tab, void *stream) {
  if (rts_status st = check_plan(plan)) return st;
  if (!mfma_precision(plan->precision)) {
    set_error("per-baseline kernels need a matrix-core plan (BF16x3 or FP32 on the matrix cores)");
    return RTS_E_UNSUPPORTED;
  }
  // replacing the tables keeps their addresses; adding or removing them would
  // leave a captured graph with the wrong kernels or freed memory
  if ((!tab || !plan->d_pb_thl) && live_graphs(plan)) {
    set_error("destroy this plan's cadence graphs before adding or removing per-baseline kernels");
    return RTS_E_INVALID;
  }
  if (!tab) {
    hipFree(plan->d_pb_thl);
    hipFree(plan->d_pb_tab);
    plan->d_pb_thl = nullptr;
    plan->d_pb_tab = nullptr;
    return RTS_OK;
  }
  RTS_REQUIRE(aligned(tab, 4), "tab must be 4-byte aligned");
  // the kernels address the tables with 32-bit word offsets
  RTS_REQUIRE(pb_table_words(*plan) < ((int64_t)1 << 32), "per-baseline tables of %d baselines exceed 2^32 words",
              plan->B);
  if (!plan->d_pb_thl) {
    const size_t words = (size_t)pb_table_words(*plan);
    RTS_HIP(dalloc(&plan->d_pb_thl, words));
    hipError_t e = dalloc(&plan->d_pb_tab, words);
    if (e != hipSuccess) {
      hipFree(plan->d_pb_thl);
      plan->d_pb_thl = nullptr;
      set_error("device allocation of %zu bytes failed", 8 * words);
      return RTS_E_NOMEM;
    }
  }
  RTS_HIP(build_baseline_tables(*plan, tab, (hipStream_t)stream));
  return RTS_OK;
}

rts_status rts_plan_get_table(rts_plan_t plan, float *tab, int64_t capacity) {
  if (rts_status st = check_plan(plan)) return st;
  RTS_REQUIRE(tab != nullptr, "tab is NULL");
  RTS_REQUIRE(capacity >= (int64_t)plan->tab.size(), "capacity %lld < %zu", (long long)capacity,
              plan->tab.size());
  std::memcpy(tab, plan->tab.data(), plan->tab.size() * sizeof(float));
  return RTS_OK;
}

rts_status rts_plan_get_info(rts_plan_t plan, rts_plan_info *info) {
  if (rts_status st = check_plan(plan)) return st;
  RTS_REQUIRE(info != nullptr, "info is NULL");
  if (plan->stats_pending) {
    unsigned long long st[8] = {0};
    RTS_HIP(hipDeviceSynchronize());
    RTS_HIP(hipMemcpy(st, plan->d_stats, sizeof st, hipMemcpyDeviceToHost));
    plan->info.n_valid = (int64_t)st[0];
    plan->info.n_flagged = (int64_t)st[1];
    plan->info.n_offgrid = (int64_t)st[2];
    plan->info.n_segments = (int64_t)st[3];
    plan->info.n_listings = (int64_t)st[4];
    plan->info.n_dropped = (int64_t)st[5];
    plan->stats_pending = false;
  }
  *info = plan->info;
  return RTS_OK;
}

rts_status rts_plan_destroy(rts_plan_t plan) {
  if (!plan) return RTS_OK;
  if (live_graphs(plan)) {
    set_error("destroy this plan's cadence graphs before the plan");
    return RTS_E_INVALID;
  }
  hipError_t e = hipDeviceSynchronize();
  free_plan(plan);
  RTS_HIP(e);
  return RTS_OK;
}

}  // extern "C"
