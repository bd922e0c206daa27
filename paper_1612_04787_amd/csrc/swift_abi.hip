// C ABI of libswift: argument validation, workspace layout and launches.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "swift_fft.hpp"
#include "swift_internal.hpp"

using namespace swift;

static_assert(sizeof(swift_image) == 32 && sizeof(swift_params) == 32 && sizeof(swift_match) == 64,
              "C ABI struct sizes");

// Records a pair of HIP events around every kernel launch while enabled.
struct EventTimer : KernelTimer {
  struct Rec {
    std::string name;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  std::string cur;
  hipEvent_t cur_a = nullptr;
  bool failed = false;
  static constexpr size_t kMaxRecs = 1 << 16;

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void begin(const char* name, int n, hipStream_t s) override {
    char buf[64];
    snprintf(buf, sizeof(buf), "%s<%d>", name, n);
    cur = buf;
    cur_a = recs.size() < kMaxRecs ? get() : nullptr;
    if (cur_a && hipEventRecord(cur_a, s) != hipSuccess) failed = true;
  }
  void end(hipStream_t s) override {
    if (!cur_a) return;
    hipEvent_t b = get();
    if (!b || hipEventRecord(b, s) != hipSuccess) {
      failed = true;
      return;
    }
    recs.push_back(Rec{cur, cur_a, b});
    cur_a = nullptr;
  }
  ~EventTimer() override {
    for (auto& r : recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// A captured and instantiated match batch, keyed by its argument tuple.
struct GraphEntry {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t last_use = 0;
};

struct swift_ctx {
  int device;
  float2* tw;  // W_1024^m = exp(-2 pi i m / 1024), then the lane-major register twiddles
  bool profile = false;
  EventTimer timer;
  KernelTimer* kt() { return profile ? &timer : nullptr; }
  // one stream per window size for concurrent size groups (default priority),
  // the fork/join events, and a capture stream for graphs
  hipStream_t gs[SWIFT_NSIZES] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[SWIFT_NSIZES] = {};
  hipStream_t cap = nullptr;
  std::map<std::string, GraphEntry> graphs;
  uint64_t tick = 0;
  // row-count variant per window size (swift_plan / swift_autotune)
  // default plan: the one-workgroup kernel at n = 64 (faster there on MI355X),
  // the five-kernel path elsewhere
  uint8_t alt_fwd[SWIFT_NSIZES] = {kFusedVariant, 0, 0, 0, 0};
  uint8_t alt_inv[SWIFT_NSIZES] = {};
  // chunks per size group: > 1 splits a group into chunks whose kernel
  // sequences run on two streams, so one chunk's row pass overlaps another's
  // column pass (created on first use)
  uint8_t chunks[SWIFT_NSIZES] = {1, 1, 1, 1, 1};
  hipStream_t cs[SWIFT_NSIZES][2] = {};
  hipEvent_t cfork[SWIFT_NSIZES] = {};
  hipEvent_t cjoin[SWIFT_NSIZES][2] = {};
  // tune cache: file path ("" for none) and this device's key in it
  std::string tune_path, tune_key;
  // device address of this GPU's fixed scratch array (swift_match_batch_noalloc)
  void* scratch = nullptr;
};

static constexpr size_t kMaxGraphs = 16;
static constexpr int kTuneSlots = SWIFT_TUNE_SLOTS;
static constexpr int kTuneRounds = 3;           // timing rounds over the slots
static constexpr float kTuneMargin = 0.02f;     // relative gain needed to leave a choice

static void ctx_release(swift_ctx* c) {
  for (auto& kv : c->graphs) {
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
  }
  c->graphs.clear();
  for (int i = 0; i < SWIFT_NSIZES; ++i) {
    if (c->gs[i]) (void)hipStreamDestroy(c->gs[i]);
    if (c->join_ev[i]) (void)hipEventDestroy(c->join_ev[i]);
    if (c->cfork[i]) (void)hipEventDestroy(c->cfork[i]);
    for (int j = 0; j < 2; ++j) {
      if (c->cs[i][j]) (void)hipStreamDestroy(c->cs[i][j]);
      if (c->cjoin[i][j]) (void)hipEventDestroy(c->cjoin[i][j]);
    }
  }
  if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  if (c->tw) (void)hipFree(c->tw);
}

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int ok() {
  g_err.clear();
  return SWIFT_OK;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(SWIFT_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Makes the context's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) return;
    ok = (prev == dev) || (hipSetDevice(dev) == hipSuccess);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// Workspace and saved-state layout of one batch.  The forward and the
// adjoint use the same workspace; its size is the larger of the two.
struct GroupLayout {
  int n = 0;
  int count = 0;
  int first = 0;  // index of the group's first pair
  // forward
  size_t z = 0, rowpart = 0, pstat = 0, invpart = 0, colsq = 0, ncc_rows = 0, ncc_var = 0, geom = 0;
  // adjoint
  size_t y = 0, dpart = 0, rpart = 0;
  // saved state (offsets into the saved buffer)
  size_t sz = 0, sps = 0, srec = 0, snb = 0;
};

struct Layout {
  size_t taper = 0;  // SWIFT_NSIZES x (tau, taper, TaperInfo)
  GroupLayout g[SWIFT_NSIZES];
  size_t fwd = 0, bwd = 0, total = 0, saved = 0;
};

// Per window size: tau[1024] float2, taper[1024] float, TaperInfo.
constexpr size_t kTaperSlot = 1024 * sizeof(float2) + 1024 * sizeof(float) + 256;


// pearson: room for the Pearson row sums and patch energies.
Layout make_layout(const swift_pairs* pairs, bool pearson = false) {
  Layout L;
  const size_t base = align256(SWIFT_NSIZES * kTaperSlot);
  L.taper = 0;
  size_t fo = base, bo = base, so = 0;
  int first = 0;
  for (int i = 0; i < SWIFT_NSIZES; ++i) {
    GroupLayout& g = L.g[i];
    g.n = kSizes[i];
    g.count = pairs->size_count[i];
    g.first = first;
    first += g.count;
    if (g.count == 0) continue;
    const size_t P = (size_t)g.count, n = (size_t)g.n;
    g.z = fo;
    fo += align256(P * n * n * sizeof(float2));
    g.rowpart = fo;
    fo += align256(P * (size_t)max(fwd_blocks_n(g.n, false), fwd_blocks_n(g.n, true)) * sizeof(RowPart));
    g.pstat = fo;
    fo += align256(P * sizeof(PairStat));
    g.invpart = fo;
    fo += align256(P * (size_t)max(inv_blocks_n(g.n, false), inv_blocks_n(g.n, true)) * sizeof(InvPart));
    g.colsq = fo;
    fo += align256(P * (n / 2 + 1) * sizeof(double));
    g.geom = fo;
    fo += align256(P * sizeof(PairGeom));
    if (pearson) {
      g.ncc_rows = fo;
      fo += align256(P * n * (n / 2 + 1) * sizeof(float2));
      g.ncc_var = fo;
      fo += align256(P * (n / 2 + 1) * (n / 2 + 1) * sizeof(float));
    }
    g.y = bo;
    bo += align256(P * n * n * sizeof(float2));
    g.dpart = bo;
    bo += align256(P * (size_t)bwd_col_blocks_n(g.n) * kDpart * sizeof(double));
    g.rpart = bo;
    bo += align256(P * (size_t)bwd_row_blocks_n(g.n) * 2 * kBwdSums * sizeof(double));
    g.sz = so;
    so += align256(P * n * n * sizeof(float2));
    g.sps = so;
    so += align256(P * sizeof(PairStat));
    g.srec = so;
    so += align256(P * sizeof(swift_match));
    g.snb = so;
    so += align256(P * 9 * sizeof(float));
  }
  L.fwd = fo;
  L.bwd = bo;
  L.total = fo > bo ? fo : bo;
  L.saved = so;
  return L;
}

int check_pairs(const swift_pairs* pairs) {
  if (!pairs) return fail(SWIFT_E_INVAL, "pairs is NULL");
  long long tot = 0;
  for (int i = 0; i < SWIFT_NSIZES; ++i) {
    if (pairs->size_count[i] < 0) return fail(SWIFT_E_INVAL, "size_count[%d] < 0", i);
    tot += pairs->size_count[i];
  }
  if (tot != pairs->n_pairs) return fail(SWIFT_E_INVAL, "n_pairs (%d) != sum(size_count) (%lld)", pairs->n_pairs, tot);
  if (pairs->n_pairs > 0 && (!pairs->img_a || !pairs->img_b || !pairs->theta_a || !pairs->theta_b))
    return fail(SWIFT_E_INVAL, "pair arrays must be non-NULL");
  return SWIFT_OK;
}

constexpr int kMaxExcludeR = 8;

int check_params(const swift_params* pr) {
  if (!pr) return fail(SWIFT_E_INVAL, "params is NULL");
  if (!(pr->p >= 0.0f && pr->p <= 1.0f)) return fail(SWIFT_E_INVAL, "p must be in [0, 1] (got %g)", pr->p);
  if (!(pr->eps_rel >= 0.0f) || !isfinite(pr->eps_rel))
    return fail(SWIFT_E_INVAL, "eps_rel must be finite and >= 0 (got %g)", pr->eps_rel);
  if (!(pr->taper_frac >= 0.0f && pr->taper_frac <= 1.0f))
    return fail(SWIFT_E_INVAL, "taper_frac must be in [0, 1] (got %g)", pr->taper_frac);
  if (pr->centroid_r != 1) return fail(SWIFT_E_UNSUPPORTED, "centroid_r must be 1 (got %d)", pr->centroid_r);
  if (pr->flags & ~(SWIFT_FLAG_CONCURRENT_SIZES | SWIFT_FLAG_JAC_TRANSLATION | SWIFT_FLAG_PEARSON))
    return fail(SWIFT_E_UNSUPPORTED, "unknown flags %#x", pr->flags);
  if (pr->max_shift < 0) return fail(SWIFT_E_INVAL, "max_shift must be >= 0 (got %d)", pr->max_shift);
  if ((pr->flags & SWIFT_FLAG_PEARSON) && pr->max_shift != 0)
    return fail(SWIFT_E_INVAL, "max_shift must be 0 with SWIFT_FLAG_PEARSON (its range is n/4)");
  if (pr->snr_exclude_r < 0 || pr->snr_exclude_r > kMaxExcludeR)
    return fail(SWIFT_E_INVAL, "snr_exclude_r must be in [0, %d] (got %d)", kMaxExcludeR, pr->snr_exclude_r);
  if ((pr->flags & SWIFT_FLAG_PEARSON) && pr->snr_exclude_r != 0)
    return fail(SWIFT_E_INVAL, "snr_exclude_r must be 0 with SWIFT_FLAG_PEARSON");
  if (pr->reserved != 0) return fail(SWIFT_E_INVAL, "params.reserved must be 0");
  return SWIFT_OK;
}

bool pearson_mode(const swift_params* pr) { return (pr->flags & SWIFT_FLAG_PEARSON) != 0; }

// The search radius restricts window edge n only when 0 < r < n/2.
bool prunes(const swift_params* pr, int n) { return pr->max_shift > 0 && pr->max_shift < n / 2; }

// Surfaces are whole only without a search radius; the Pearson mode keeps
// neither surfaces nor adjoint state.
int check_surfaces(const swift_pairs* pairs, const swift_params* pr, const float* surfaces, const void* saved) {
  if (pearson_mode(pr) && (surfaces || saved))
    return fail(SWIFT_E_INVAL, "surfaces and saved must be NULL with SWIFT_FLAG_PEARSON");
  if (!surfaces) return SWIFT_OK;
  for (int i = 0; i < SWIFT_NSIZES; ++i)
    if (pairs->size_count[i] > 0 && prunes(pr, kSizes[i]))
      return fail(SWIFT_E_INVAL, "surfaces must be NULL with max_shift %d (window edge %d)", pr->max_shift,
                  kSizes[i]);
  return SWIFT_OK;
}

}  // namespace

// Lane-major register twiddles of size N, copied from the W_1024 table.
template <int N>
static void fill_lane_twiddles(float2* host) {
  for (int t = 0; t < FftCfg<N>::T; ++t) {
    float2* row = host + twl_off(N) + t * tw_pad<N>();
    for (int i = 0; i < tw_pad<N>(); ++i) row[i] = i < tw_count<N>() ? host[tw_index<N>(t, i)] : make_float2(0.f, 0.f);
  }
}

static bool valid_chunks(int c) { return c == 1 || c == 2 || c == 4 || c == 8; }

// ---------------------------------------------------------------- fixed scratch
// Workspace of swift_match_batch_noalloc: a file-scope device array, one per
// GPU the library runs on, held until the process ends.  Host code uses its
// device address, read once per device by swift_create.
constexpr size_t kScratchBytes = SWIFT_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static void* g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// With `device` current: the device address of this GPU's scratch array.
static hipError_t scratch_address(int device, void** ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}

// ---------------------------------------------------------------- tune cache
// A text file of plan lines "<device key> <n> <fwd variant> <inv variant>",
// one per device and window size; '#' starts a comment.  The device key is
// the architecture name and the compute-unit count, so a file can serve
// several kinds of device.
static std::string device_key(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string arch(prop.gcnArchName);
  for (char& ch : arch)
    if (ch == ' ' || ch == '\t') ch = '_';
  char buf[320];
  snprintf(buf, sizeof(buf), "%s/cu%d", arch.c_str(), prop.multiProcessorCount);
  return buf;
}

static void tune_cache_load(swift_ctx* c) {
  FILE* f = fopen(c->tune_path.c_str(), "r");
  if (!f) return;
  char line[512], key[320];
  int n, vf, vi, ch;
  while (fgets(line, sizeof(line), f)) {
    if (line[0] == '#') continue;
    const int got = sscanf(line, "%319s %d %d %d %d", key, &n, &vf, &vi, &ch);
    if (got < 4) continue;
    if (got == 4) ch = 1;
    const int vf_max = n <= kFusedMaxN ? kFusedVariant : 1;
    if (c->tune_key != key || vf < 0 || vf > vf_max || vi < 0 || vi > 1 || !valid_chunks(ch)) continue;
    for (int i = 0; i < SWIFT_NSIZES; ++i)
      if (kSizes[i] == n) {
        c->alt_fwd[i] = (uint8_t)vf;
        c->alt_inv[i] = (uint8_t)vi;
        c->chunks[i] = (uint8_t)ch;
      }
  }
  fclose(f);
}

// Rewrites the file: other devices' lines (and this device's sizes not in
// `tuned`) are kept, this device's tuned sizes get the context's plan.
static bool tune_cache_store(const swift_ctx* c, const bool (&tuned)[SWIFT_NSIZES]) {
  std::vector<std::string> keep;
  if (FILE* f = fopen(c->tune_path.c_str(), "r")) {
    char line[512], key[320];
    int n;
    while (fgets(line, sizeof(line), f)) {
      if (line[0] == '#') continue;
      if (sscanf(line, "%319s %d", key, &n) == 2 && c->tune_key == key) {
        bool mine = false;
        for (int i = 0; i < SWIFT_NSIZES; ++i) mine |= tuned[i] && kSizes[i] == n;
        if (mine) continue;
      }
      std::string l(line);
      if (!l.empty() && l.back() != '\n') l += '\n';
      keep.push_back(l);
    }
    fclose(f);
  }
  const std::string tmp = c->tune_path + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return false;
  bool good = fputs("# libswift tune cache: <device> <n> <fwd variant> <inv variant> <chunks>\n", f) >= 0;
  for (const auto& l : keep) good = good && fputs(l.c_str(), f) >= 0;
  for (int i = 0; i < SWIFT_NSIZES; ++i)
    if (tuned[i])
      good = good && fprintf(f, "%s %d %d %d %d\n", c->tune_key.c_str(), kSizes[i], c->alt_fwd[i], c->alt_inv[i],
                             c->chunks[i]) > 0;
  good = (fclose(f) == 0) && good;
  return good && rename(tmp.c_str(), c->tune_path.c_str()) == 0;
}

extern "C" {

const char* swift_last_error(void) { return g_err.c_str(); }

int swift_create(int device, const char* tune_cache_path, swift_ctx** out) {
  if (!out) return fail(SWIFT_E_INVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= ndev) return fail(SWIFT_E_INVAL, "device %d out of range (%d devices)", device, ndev);
  DeviceGuard dg(device);
  if (!dg.ok) return fail(SWIFT_E_HIP, "cannot select device %d", device);
  std::vector<float2> host(kTwTotal);
  for (int m = 0; m < 1024; ++m) {
    const double a = -2.0 * M_PI * (double)m / 1024.0;
    host[m] = make_float2((float)cos(a), (float)sin(a));
  }
  fill_lane_twiddles<64>(host.data());
  fill_lane_twiddles<128>(host.data());
  fill_lane_twiddles<256>(host.data());
  fill_lane_twiddles<512>(host.data());
  fill_lane_twiddles<1024>(host.data());
  float2* tw = nullptr;
  e = hipMalloc((void**)&tw, host.size() * sizeof(float2));
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(twiddles)");
  e = hipMemcpy(tw, host.data(), host.size() * sizeof(float2), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(tw);
    return hip_fail(e, "hipMemcpy(twiddles)");
  }
  swift_ctx* c = new (std::nothrow) swift_ctx;
  if (!c) {
    (void)hipFree(tw);
    return fail(SWIFT_E_INVAL, "out of host memory");
  }
  c->device = device;
  c->tw = tw;
  for (int i = 0; i < SWIFT_NSIZES && e == hipSuccess; ++i) {
    e = hipStreamCreateWithFlags(&c->gs[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->join_ev[i], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
  if (e != hipSuccess) {
    ctx_release(c);
    delete c;
    return hip_fail(e, "context streams/events");
  }
  e = scratch_address(device, &c->scratch);
  if (e != hipSuccess) {
    ctx_release(c);
    delete c;
    return hip_fail(e, "hipGetSymbolAddress(scratch)");
  }
  if (tune_cache_path && tune_cache_path[0]) {
    c->tune_path = tune_cache_path;
    c->tune_key = device_key(device);
    tune_cache_load(c);
  }
  *out = c;
  return ok();
}

void swift_destroy(swift_ctx* ctx) {
  if (!ctx) return;
  DeviceGuard dg(ctx->device);
  (void)hipDeviceSynchronize();
  ctx_release(ctx);
  delete ctx;
}

int swift_workspace_size(swift_ctx* ctx, const swift_pairs* pairs, const swift_params* params, size_t* ws_bytes,
                         size_t* saved_bytes) {
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  if (!ws_bytes) return fail(SWIFT_E_INVAL, "ws_bytes is NULL");
  int rc = check_pairs(pairs);
  if (rc) return rc;
  rc = check_params(params);
  if (rc) return rc;
  const Layout L = make_layout(pairs, pearson_mode(params));
  *ws_bytes = L.total;
  if (saved_bytes) *saved_bytes = L.saved;
  return ok();
}

// Validation shared by swift_match_batch and swift_match_graph; sets *empty
// for a batch without pairs.
static int check_match(swift_ctx* ctx, const swift_image* imgs, int32_t n_imgs, const swift_pairs* pairs,
                       const swift_params* params, swift_match* out, void* ws, size_t ws_bytes, bool* empty) {
  *empty = false;
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  int rc = check_pairs(pairs);
  if (rc) return rc;
  rc = check_params(params);
  if (rc) return rc;
  if (pairs->n_pairs == 0) {
    *empty = true;
    return ok();
  }
  if (!imgs || n_imgs <= 0) return fail(SWIFT_E_INVAL, "image table is empty");
  if (!out) return fail(SWIFT_E_INVAL, "out is NULL");
  const Layout L = make_layout(pairs, pearson_mode(params));
  if (!ws || ws_bytes < L.total)
    return fail(SWIFT_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", L.total, ws ? ws_bytes : (size_t)0);
  return SWIFT_OK;
}

// The size group of `a` as nch chunks of consecutive pairs, alternating
// between the context's two chunk streams of size i (forked from and joined
// back into s).  Every per-pair array of a chunk is the group's array from
// its first pair on, so the chunks' results are those of one launch.
static int enqueue_chunks(swift_ctx* ctx, int i, const GroupLayout& g, const MatchArgs& a, int nch, hipStream_t s,
                          KernelTimer* kt) {
  hipError_t e = hipSuccess;
  for (int j = 0; j < 2 && e == hipSuccess; ++j) {
    if (!ctx->cs[i][j]) e = hipStreamCreateWithFlags(&ctx->cs[i][j], hipStreamNonBlocking);
    if (e == hipSuccess && !ctx->cjoin[i][j]) e = hipEventCreateWithFlags(&ctx->cjoin[i][j], hipEventDisableTiming);
  }
  if (e == hipSuccess && !ctx->cfork[i]) e = hipEventCreateWithFlags(&ctx->cfork[i], hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(ctx->cfork[i], s);
  for (int j = 0; j < 2 && e == hipSuccess; ++j) e = hipStreamWaitEvent(ctx->cs[i][j], ctx->cfork[i], 0);
  if (e != hipSuccess) return hip_fail(e, "chunk fork");
  const size_t n = (size_t)g.n, P = (size_t)g.count;
  const int af = ctx->alt_fwd[i];
  const bool ai = ctx->alt_inv[i] != 0;
  for (int c = 0; c < nch; ++c) {
    const size_t p0 = P * c / nch, p1 = P * (c + 1) / nch;
    MatchArgs b = a;
    b.npairs = (int)(p1 - p0);
    b.img_a += p0;
    b.img_b += p0;
    b.th_a += 8 * p0;
    b.th_b += 8 * p0;
    b.out += p0;
    if (b.surfaces) b.surfaces += p0 * n * n;
    b.Z += p0 * n * n;
    b.rowpart += p0 * (size_t)a.nsl_fwd;
    b.pstat += p0;
    b.geom += p0;
    b.invpart += p0 * (size_t)a.nsl_inv;
    b.colsq += p0 * (n / 2 + 1);
    if (b.ncc_rows) b.ncc_rows += p0 * n * (n / 2 + 1);
    if (b.ncc_var) b.ncc_var += p0 * (n / 2 + 1) * (n / 2 + 1);
    if (b.saved_Z) b.saved_Z += p0 * n * n;
    if (b.saved_ps) b.saved_ps += p0;
    if (b.saved_rec) b.saved_rec += p0;
    if (b.saved_nb) b.saved_nb += 9 * p0;
    e = launch_match_group(g.n, b, af, ai, ctx->cs[i][c & 1], kt);
    if (e != hipSuccess) return hip_fail(e, "match launch");
  }
  for (int j = 0; j < 2 && e == hipSuccess; ++j) {
    e = hipEventRecord(ctx->cjoin[i][j], ctx->cs[i][j]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, ctx->cjoin[i][j], 0);
  }
  if (e != hipSuccess) return hip_fail(e, "chunk join");
  return SWIFT_OK;
}

// A size group whose forward row pass launches at least this many
// workgroups (32 per CU) keeps the whole GPU busy by itself: running it beside
// other groups only makes them share the CUs.
constexpr long long kFillBlocks = 8192;

// Enqueues the whole batch on `stream`: per size group the taper tables and
// the five match kernels.  With `concurrent` and more than one group, each
// group too small to fill the GPU runs on the context's stream for its size,
// forked from `stream` by an event and joined back into it; the others run on
// `stream` itself, one after another.
static int enqueue_match(swift_ctx* ctx, const swift_image* imgs, int32_t n_imgs, const swift_pairs* pairs,
                         const swift_params* params, swift_match* out, float* surfaces, void* saved, void* ws,
                         hipStream_t stream, bool concurrent, KernelTimer* kt, bool allow_chunks = true) {
  const bool pearson = pearson_mode(params);
  const Layout L = make_layout(pairs, pearson);
  bool side[SWIFT_NSIZES];
  int groups = 0, small = 0;
  for (int i = 0; i < SWIFT_NSIZES; ++i) {
    groups += L.g[i].count > 0 ? 1 : 0;
    const long long blocks = (long long)L.g[i].count * fwd_blocks_n(L.g[i].n, ctx->alt_fwd[i] == 1);
    side[i] = L.g[i].count > 0 && blocks < kFillBlocks;
    small += side[i] ? 1 : 0;
  }
  // a single group, or only groups that fill the GPU: nothing runs beside them
  concurrent = concurrent && groups > 1 && small > 0;
  if (!concurrent)
    for (int i = 0; i < SWIFT_NSIZES; ++i) side[i] = false;
  hipError_t e = hipSuccess;
  if (concurrent) {
    e = hipEventRecord(ctx->fork_ev, stream);
    if (e != hipSuccess) return hip_fail(e, "fork event");
  }
  char* base = (char*)ws;
  // surfaces are laid out by ascending window size; the groups are launched
  // longest first (LPT order, work ~ pairs x n^2 log2 n), which matters when
  // they run as concurrent branches
  size_t surf_at[SWIFT_NSIZES];
  int order[SWIFT_NSIZES];
  {
    size_t off = 0;
    for (int i = 0; i < SWIFT_NSIZES; ++i) {
      surf_at[i] = off;
      off += (size_t)L.g[i].count * L.g[i].n * L.g[i].n;
      order[i] = i;
    }
    auto work = [&](int i) { return (double)L.g[i].count * L.g[i].n * L.g[i].n * log2((double)L.g[i].n); };
    for (int i = 1; i < SWIFT_NSIZES; ++i)
      for (int j = i; j > 0 && work(order[j]) > work(order[j - 1]); --j) {
        const int t = order[j];
        order[j] = order[j - 1];
        order[j - 1] = t;
      }
  }
  for (int oi = 0; oi < SWIFT_NSIZES; ++oi) {
    const int i = order[oi];
    const GroupLayout& g = L.g[i];
    if (g.count == 0) continue;
    const size_t surf_off = surf_at[i];
    hipStream_t s = stream;
    if (side[i]) {
      s = ctx->gs[i];
      e = hipStreamWaitEvent(s, ctx->fork_ev, 0);
      if (e != hipSuccess) return hip_fail(e, "fork wait");
    }
    float2* tau = (float2*)(base + L.taper + i * kTaperSlot);
    float* taper = (float*)(base + L.taper + i * kTaperSlot + 1024 * sizeof(float2));
    TaperInfo* tinfo = (TaperInfo*)(base + L.taper + i * kTaperSlot + 1024 * sizeof(float2) + 1024 * sizeof(float));
    e = launch_taper(g.n, params->taper_frac, tau, taper, tinfo, s, pearson);
    if (e != hipSuccess) return hip_fail(e, "taper launch");
    MatchArgs a;
    a.imgs = imgs;
    a.n_imgs = n_imgs;
    a.img_a = pairs->img_a + g.first;
    a.img_b = pairs->img_b + g.first;
    a.th_a = pairs->theta_a + 8 * (size_t)g.first;
    a.th_b = pairs->theta_b + 8 * (size_t)g.first;
    a.out = out + g.first;
    a.surfaces = surfaces ? surfaces + surf_off : nullptr;
    a.Z = (float2*)(base + g.z);
    a.rowpart = (RowPart*)(base + g.rowpart);
    a.pstat = (PairStat*)(base + g.pstat);
    a.invpart = (InvPart*)(base + g.invpart);
    a.geom = (PairGeom*)(base + g.geom);
    a.tw = ctx->tw;
    a.tau = tau;
    a.taper = taper;
    a.tinfo = tinfo;
    a.p = params->p;
    a.eps_rel = params->eps_rel;
    a.L = (int)floor((double)params->taper_frac * g.n / 2.0 + 0.5);
    a.snr_exclude_r = pearson ? 0 : params->snr_exclude_r;
    a.npairs = g.count;
    a.nsl_fwd = fwd_blocks_n(g.n, ctx->alt_fwd[i] == 1);
    a.nsl_inv = inv_blocks_n(g.n, ctx->alt_inv[i] != 0);
    a.colsq = (double*)(base + g.colsq);
    a.max_shift = 0;
    a.nsl_lo = a.nsl_inv;
    a.zlo = a.zhi = g.n;
    a.pearson = pearson ? 1 : 0;
    a.ncc_rows = pearson ? (float2*)(base + g.ncc_rows) : nullptr;
    a.ncc_var = pearson ? (float*)(base + g.ncc_var) : nullptr;
    if (pearson) a.p = 0.0f;
    const int radius = pearson ? g.n / 4 : params->max_shift;
    if (radius > 0 && radius < g.n / 2) {
      // rows |y| <= r + 1 (the centroid reads one row past the window),
      // rounded out to whole inverse row blocks of R2 rows
      // (and the rows of a wider background box, whose sums k_finalize needs)
      const int full = a.nsl_inv, R2 = g.n / full;
      const int rr = radius + (params->snr_exclude_r > 1 ? params->snr_exclude_r : 1);
      const int lo = rr / R2 + 1, hs = (g.n - rr) / R2;
      a.max_shift = radius;
      if (lo < hs) {
        a.nsl_lo = lo;
        a.nsl_inv = lo + (full - hs);
        a.zlo = lo * R2;
        a.zhi = hs * R2;
      }
    }
    a.saved_Z = saved ? (float2*)((char*)saved + g.sz) : nullptr;
    a.saved_ps = saved ? (PairStat*)((char*)saved + g.sps) : nullptr;
    a.saved_rec = saved ? (swift_match*)((char*)saved + g.srec) : nullptr;
    a.saved_nb = saved ? (float*)((char*)saved + g.snb) : nullptr;
    // chunks split one group's passes over two streams; in a call whose
    // groups run concurrently no group is split (also not those on the call's
    // stream)
    const int nch = (allow_chunks && !concurrent) ? min((int)ctx->chunks[i], g.count) : 1;
    if (nch <= 1) {
      e = launch_match_group(g.n, a, ctx->alt_fwd[i], ctx->alt_inv[i] != 0, s, kt);
      if (e != hipSuccess) return hip_fail(e, "match launch");
    } else {
      const int rc = enqueue_chunks(ctx, i, g, a, nch, s, kt);
      if (rc) return rc;
    }
    if (side[i]) {
      e = hipEventRecord(ctx->join_ev[i], s);
      if (e == hipSuccess) e = hipStreamWaitEvent(stream, ctx->join_ev[i], 0);
      if (e != hipSuccess) return hip_fail(e, "join");
    }
  }
  return ok();
}

int swift_match_batch(swift_ctx* ctx, const swift_image* imgs, int32_t n_imgs, const swift_pairs* pairs,
                      const swift_params* params, swift_match* out, float* surfaces, void* saved, void* ws,
                      size_t ws_bytes, hipStream_t stream) {
  bool empty;
  int rc = check_match(ctx, imgs, n_imgs, pairs, params, out, ws, ws_bytes, &empty);
  if (rc || empty) return rc;
  rc = check_surfaces(pairs, params, surfaces, saved);
  if (rc) return rc;
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(SWIFT_E_HIP, "cannot select device %d", ctx->device);
  return enqueue_match(ctx, imgs, n_imgs, pairs, params, out, surfaces, saved, ws, stream,
                       (params->flags & SWIFT_FLAG_CONCURRENT_SIZES) != 0, ctx->kt());
}

int swift_match_batch_noalloc(swift_ctx* ctx, const swift_image* imgs, int32_t n_imgs, const swift_pairs* pairs,
                              const swift_params* params, swift_match* out, hipStream_t stream) {
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  int rc = check_pairs(pairs);
  if (rc) return rc;
  rc = check_params(params);
  if (rc) return rc;
  if (pairs->n_pairs == 0) return ok();
  if (!imgs || n_imgs <= 0) return fail(SWIFT_E_INVAL, "image table is empty");
  if (!out) return fail(SWIFT_E_INVAL, "out is NULL");
  const Layout L = make_layout(pairs, pearson_mode(params));
  if (L.total > kScratchBytes)
    return fail(SWIFT_E_WORKSPACE, "batch needs %zu bytes of workspace; the fixed scratch holds %zu", L.total,
                kScratchBytes);
  if (!ctx->scratch) return fail(SWIFT_E_HIP, "no scratch address for device %d", ctx->device);
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(SWIFT_E_HIP, "cannot select device %d", ctx->device);
  // one stream, one launch sequence per size group, no kernel timing: nothing
  // is created or allocated
  return enqueue_match(ctx, imgs, n_imgs, pairs, params, out, nullptr, nullptr, ctx->scratch, stream, false,
                       nullptr, false);
}

int swift_match_graph(swift_ctx* ctx, const swift_image* imgs, int32_t n_imgs, const swift_pairs* pairs,
                      const swift_params* params, swift_match* out, float* surfaces, void* saved, void* ws,
                      size_t ws_bytes, hipStream_t stream) {
  bool empty;
  int rc = check_match(ctx, imgs, n_imgs, pairs, params, out, ws, ws_bytes, &empty);
  if (rc || empty) return rc;
  rc = check_surfaces(pairs, params, surfaces, saved);
  if (rc) return rc;
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(SWIFT_E_HIP, "cannot select device %d", ctx->device);
  // key: every value the captured launches bake in
  struct {
    const void* p[9];
    int32_t n_imgs, n_pairs, counts[SWIFT_NSIZES];
    swift_params prm;
    uint8_t plan[3 * SWIFT_NSIZES];
  } key;
  memset(&key, 0, sizeof(key));
  key.p[0] = imgs;
  key.p[1] = pairs->img_a;
  key.p[2] = pairs->img_b;
  key.p[3] = pairs->theta_a;
  key.p[4] = pairs->theta_b;
  key.p[5] = out;
  key.p[6] = surfaces;
  key.p[7] = saved;
  key.p[8] = ws;
  key.n_imgs = n_imgs;
  key.n_pairs = pairs->n_pairs;
  for (int i = 0; i < SWIFT_NSIZES; ++i) key.counts[i] = pairs->size_count[i];
  key.prm = *params;
  for (int i = 0; i < SWIFT_NSIZES; ++i) {
    key.plan[i] = ctx->alt_fwd[i];
    key.plan[SWIFT_NSIZES + i] = ctx->alt_inv[i];
    key.plan[2 * SWIFT_NSIZES + i] = ctx->chunks[i];
  }
  const std::string k((const char*)&key, sizeof(key));
  auto it = ctx->graphs.find(k);
  if (it == ctx->graphs.end()) {
    if (ctx->graphs.size() >= kMaxGraphs) {  // evict the least recently used
      auto lru = ctx->graphs.begin();
      for (auto j = ctx->graphs.begin(); j != ctx->graphs.end(); ++j)
        if (j->second.last_use < lru->second.last_use) lru = j;
      (void)hipGraphExecDestroy(lru->second.exec);
      (void)hipGraphDestroy(lru->second.graph);
      ctx->graphs.erase(lru);
    }
    GraphEntry ge;
    hipError_t e = hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(SWIFT_E_CAPTURE, "begin capture: %s", hipGetErrorString(e));
    rc = enqueue_match(ctx, imgs, n_imgs, pairs, params, out, surfaces, saved, ws, ctx->cap, true, nullptr);
    e = hipStreamEndCapture(ctx->cap, &ge.graph);
    if (rc) {
      if (ge.graph) (void)hipGraphDestroy(ge.graph);
      return rc;
    }
    if (e != hipSuccess) return fail(SWIFT_E_CAPTURE, "end capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&ge.exec, ge.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(ge.graph);
      return fail(SWIFT_E_CAPTURE, "instantiate: %s", hipGetErrorString(e));
    }
    it = ctx->graphs.emplace(k, ge).first;
  }
  it->second.last_use = ++ctx->tick;
  hipError_t e = hipGraphLaunch(it->second.exec, stream);
  if (e != hipSuccess) return fail(SWIFT_E_CAPTURE, "graph launch: %s", hipGetErrorString(e));
  return ok();
}

// Shared body of the two adjoint entry points: per size group, the taper
// tables and one backward launch (centroid_jac selects the objective).
static int run_backward(swift_ctx* ctx, const swift_image* imgs, int32_t n_imgs, const swift_pairs* pairs,
                        const swift_params* params, const void* saved, const float* g_peak, const float* g_snr,
                        float* g_theta_a, float* g_theta_b, float* peak_hess, float* jac, void* ws,
                        size_t ws_bytes, hipStream_t stream) {
  const bool cj = jac != nullptr;
  if (pearson_mode(params))
    return fail(SWIFT_E_UNSUPPORTED, "the adjoint of the Pearson-normalised match is not implemented");
  const Layout L = make_layout(pairs);
  if (!ws || ws_bytes < L.total)
    return fail(SWIFT_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", L.total, ws ? ws_bytes : (size_t)0);
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(SWIFT_E_HIP, "cannot select device %d", ctx->device);
  char* base = (char*)ws;
  for (int i = 0; i < SWIFT_NSIZES; ++i) {
    const GroupLayout& g = L.g[i];
    if (g.count == 0) continue;
    float2* tau = (float2*)(base + L.taper + i * kTaperSlot);
    float* taper = (float*)(base + L.taper + i * kTaperSlot + 1024 * sizeof(float2));
    TaperInfo* tinfo = (TaperInfo*)(base + L.taper + i * kTaperSlot + 1024 * sizeof(float2) + 1024 * sizeof(float));
    hipError_t e = launch_taper(g.n, params->taper_frac, tau, taper, tinfo, stream);
    if (e != hipSuccess) return hip_fail(e, "taper launch");
    BwdArgs b;
    b.imgs = imgs;
    b.n_imgs = n_imgs;
    b.img_a = pairs->img_a + g.first;
    b.img_b = pairs->img_b + g.first;
    b.th_a = pairs->theta_a + 8 * (size_t)g.first;
    b.th_b = pairs->theta_b + 8 * (size_t)g.first;
    b.Zf = (const float2*)((const char*)saved + g.sz);
    b.ps = (const PairStat*)((const char*)saved + g.sps);
    b.rec = (const swift_match*)((const char*)saved + g.srec);
    b.nb = (const float*)((const char*)saved + g.snb);
    b.g_peak = g_peak ? g_peak + g.first : nullptr;
    b.g_snr = g_snr ? g_snr + g.first : nullptr;
    b.g_th_a = g_theta_a ? g_theta_a + 6 * (size_t)g.first : nullptr;
    b.g_th_b = g_theta_b ? g_theta_b + 6 * (size_t)g.first : nullptr;
    b.peak_hess = peak_hess ? peak_hess + 3 * (size_t)g.first : nullptr;
    b.jac = jac ? jac + 12 * (size_t)g.first : nullptr;
    b.Y = (float2*)(base + g.y);
    b.dpart = (double*)(base + g.dpart);
    b.rpart = (double*)(base + g.rpart);
    b.tw = ctx->tw;
    b.tau = tau;
    b.taper = taper;
    b.tinfo = tinfo;
    b.p = params->p;
    b.eps_rel = params->eps_rel;
    b.L = (int)floor((double)params->taper_frac * g.n / 2.0 + 0.5);
    b.npairs = g.count;
    b.jac_trans = (cj && (params->flags & SWIFT_FLAG_JAC_TRANSLATION)) ? 1 : 0;
    e = launch_backward_group(g.n, b, cj, stream, ctx->kt());
    if (e != hipSuccess) return hip_fail(e, "backward launch");
  }
  return ok();
}

static int check_backward_common(swift_ctx* ctx, const swift_image* imgs, int32_t n_imgs, const swift_pairs* pairs,
                                 const swift_params* params, const void* saved, bool* empty) {
  *empty = false;
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  int rc = check_pairs(pairs);
  if (rc) return rc;
  rc = check_params(params);
  if (rc) return rc;
  if (params->snr_exclude_r != 0)
    return fail(SWIFT_E_UNSUPPORTED, "the adjoint takes the whole surface as the SNR background (snr_exclude_r 0)");
  if (pairs->n_pairs == 0) {
    *empty = true;
    return ok();
  }
  if (!imgs || n_imgs <= 0) return fail(SWIFT_E_INVAL, "image table is empty");
  if (!saved) return fail(SWIFT_E_INVAL, "saved is NULL (run swift_match_batch with a saved buffer first)");
  return ok();
}

int swift_match_backward(swift_ctx* ctx, const swift_image* imgs, int32_t n_imgs, const swift_pairs* pairs,
                         const swift_params* params, const void* saved, const float* g_peak, const float* g_snr,
                         float* g_theta_a, float* g_theta_b, float* peak_hess, void* ws, size_t ws_bytes,
                         hipStream_t stream) {
  bool empty;
  int rc = check_backward_common(ctx, imgs, n_imgs, pairs, params, saved, &empty);
  if (rc || empty) return rc;
  if (!g_theta_a) return fail(SWIFT_E_INVAL, "g_theta_a is NULL");
  return run_backward(ctx, imgs, n_imgs, pairs, params, saved, g_peak, g_snr, g_theta_a, g_theta_b, peak_hess,
                      nullptr, ws, ws_bytes, stream);
}

int swift_centroid_jacobian(swift_ctx* ctx, const swift_image* imgs, int32_t n_imgs, const swift_pairs* pairs,
                            const swift_params* params, const void* saved, float* jac, void* ws, size_t ws_bytes,
                            hipStream_t stream) {
  bool empty;
  int rc = check_backward_common(ctx, imgs, n_imgs, pairs, params, saved, &empty);
  if (rc || empty) return rc;
  if (!jac) return fail(SWIFT_E_INVAL, "jac is NULL");
  return run_backward(ctx, imgs, n_imgs, pairs, params, saved, nullptr, nullptr, nullptr, nullptr, nullptr, jac,
                      ws, ws_bytes, stream);
}

int swift_project(swift_ctx* ctx, const uint8_t* stack, int32_t S, int32_t height, int32_t width, int64_t pitch,
                  int64_t section_stride, const uint8_t* exclude, int32_t k, uint8_t* out, int64_t out_pitch,
                  int64_t out_section_stride, hipStream_t stream) {
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  if (!stack || !out) return fail(SWIFT_E_INVAL, "stack/out is NULL");
  if (S < 1 || height < 1 || width < 1) return fail(SWIFT_E_INVAL, "bad stack shape %d x %d x %d", S, height, width);
  if (k < 1 || k > 8) return fail(SWIFT_E_INVAL, "k must be in [1, 8] (got %d)", k);
  if (pitch < width || out_pitch < width) return fail(SWIFT_E_INVAL, "pitch smaller than width");
  if (section_stride < pitch * height || out_section_stride < out_pitch * height)
    return fail(SWIFT_E_INVAL, "section stride smaller than height * pitch");
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(SWIFT_E_HIP, "cannot select device %d", ctx->device);
  hipError_t e = launch_project(stack, pitch, section_stride, S, height, width, exclude, k, out, out_pitch,
                                out_section_stride, stream, ctx->kt());
  if (e != hipSuccess) return hip_fail(e, "project launch");
  return ok();
}

int swift_project_side(swift_ctx* ctx, const uint8_t* stack, int32_t S, int32_t height, int32_t width, int64_t pitch,
                       int64_t section_stride, const uint8_t* exclude, int32_t k, int32_t side, uint8_t* out,
                       int64_t out_pitch, int64_t out_section_stride, hipStream_t stream) {
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  if (side != -1 && side != 1) return fail(SWIFT_E_INVAL, "side must be -1 or +1 (got %d)", side);
  if (!stack || !out) return fail(SWIFT_E_INVAL, "stack/out is NULL");
  if (S < 1 || height < 1 || width < 1) return fail(SWIFT_E_INVAL, "bad stack shape %d x %d x %d", S, height, width);
  if (k < 1 || k > 8) return fail(SWIFT_E_INVAL, "k must be in [1, 8] (got %d)", k);
  if (pitch < width || out_pitch < width) return fail(SWIFT_E_INVAL, "pitch smaller than width");
  if (section_stride < pitch * height || out_section_stride < out_pitch * height)
    return fail(SWIFT_E_INVAL, "section stride smaller than height * pitch");
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(SWIFT_E_HIP, "cannot select device %d", ctx->device);
  hipError_t e = launch_project(stack, pitch, section_stride, S, height, width, exclude, k, out, out_pitch,
                                out_section_stride, stream, ctx->kt(), side);
  if (e != hipSuccess) return hip_fail(e, "one-sided project launch");
  return ok();
}

int swift_blend_span(swift_ctx* ctx, int32_t S, int32_t a, int32_t b, const double* aff_left,
                     const double* aff_right, double* aff, hipStream_t stream) {
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  if (!aff_left || !aff_right || !aff) return fail(SWIFT_E_INVAL, "NULL affine array");
  if (!(0 <= a && a <= b && b < S)) return fail(SWIFT_E_INVAL, "span [%d, %d] outside [0, %d)", a, b, S);
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(SWIFT_E_HIP, "cannot select device %d", ctx->device);
  hipError_t e = launch_blend_span(a, b, aff_left, aff_right, aff, stream);
  if (e != hipSuccess) return hip_fail(e, "blend launch");
  return ok();
}

int swift_join_break(swift_ctx* ctx, int32_t S, int32_t j, const double* aff, const double* aff_left, double* out,
                     hipStream_t stream) {
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  if (!aff || !aff_left || !out) return fail(SWIFT_E_INVAL, "NULL affine array");
  if (aff == out) return fail(SWIFT_E_INVAL, "out must not alias aff");
  if (!(0 <= j && j < S)) return fail(SWIFT_E_INVAL, "break %d outside [0, %d)", j, S);
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(SWIFT_E_HIP, "cannot select device %d", ctx->device);
  hipError_t e = launch_join_break(S, j, aff, aff_left, out, stream);
  if (e != hipSuccess) return hip_fail(e, "join launch");
  return ok();
}

int swift_search_keep(swift_ctx* ctx, int32_t P, int32_t n, const int32_t* idx, const swift_match* recs,
                      int32_t cand, float accept, swift_match* best, int32_t* best_cand, uint8_t* done,
                      hipStream_t stream) {
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  if (P < 0 || n < 0 || n > P) return fail(SWIFT_E_INVAL, "bad sizes (P %d, n %d)", P, n);
  if (n > 0 && (!idx || !recs || !best || !best_cand || !done)) return fail(SWIFT_E_INVAL, "NULL array");
  if (cand < 0) return fail(SWIFT_E_INVAL, "cand must be >= 0 (got %d)", cand);
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(SWIFT_E_HIP, "cannot select device %d", ctx->device);
  hipError_t e = launch_search_keep(P, n, idx, recs, cand, accept, best, best_cand, done, stream);
  if (e != hipSuccess) return hip_fail(e, "search launch");
  return ok();
}

int swift_search_next(swift_ctx* ctx, int32_t P, const uint8_t* done, float ox, float oy, const int32_t* img_a,
                      const int32_t* img_b, const float* theta_a, const float* theta_b, int32_t* idx,
                      int32_t* img_a_out, int32_t* img_b_out, float* theta_a_out, float* theta_b_out,
                      int32_t* count, hipStream_t stream) {
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  if (P < 0) return fail(SWIFT_E_INVAL, "bad size (P %d)", P);
  if (!count) return fail(SWIFT_E_INVAL, "count is NULL");
  if (P > 0 && (!done || !img_a || !img_b || !theta_a || !theta_b || !idx || !img_a_out || !img_b_out ||
                !theta_a_out || !theta_b_out))
    return fail(SWIFT_E_INVAL, "NULL array");
  if (P > 0 && (theta_a_out == theta_a || theta_b_out == theta_b || img_a_out == img_a || img_b_out == img_b))
    return fail(SWIFT_E_INVAL, "outputs must not alias the inputs");
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(SWIFT_E_HIP, "cannot select device %d", ctx->device);
  hipError_t e = launch_search_next(P, done, ox, oy, img_a, img_b, theta_a, theta_b, idx, img_a_out, img_b_out,
                                    theta_a_out, theta_b_out, count, stream);
  if (e != hipSuccess) return hip_fail(e, "search gather launch");
  return ok();
}

int swift_pyramid(swift_ctx* ctx, const swift_image* src, const swift_image* dst, hipStream_t stream) {
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  if (!src || !dst || !src->data || !dst->data) return fail(SWIFT_E_INVAL, "src/dst is NULL");
  if (src->dtype != SWIFT_U8 || dst->dtype != SWIFT_U8) return fail(SWIFT_E_UNSUPPORTED, "pyramid needs uint8 images");
  if (src->width < 2 || src->height < 2) return fail(SWIFT_E_INVAL, "source smaller than 2 x 2");
  if (dst->width != src->width / 2 || dst->height != src->height / 2)
    return fail(SWIFT_E_INVAL, "destination must be %d x %d", src->width / 2, src->height / 2);
  if (src->pitch < src->width || dst->pitch < dst->width) return fail(SWIFT_E_INVAL, "pitch smaller than width");
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(SWIFT_E_HIP, "cannot select device %d", ctx->device);
  hipError_t e = launch_pyramid((const uint8_t*)src->data, src->pitch, src->width, src->height, (uint8_t*)dst->data,
                                dst->pitch, dst->width, dst->height, stream);
  if (e != hipSuccess) return hip_fail(e, "pyramid launch");
  return ok();
}

int swift_snr(swift_ctx* ctx, const float* surfaces, int32_t n, int32_t batch, const swift_params* params,
              swift_match* out, hipStream_t stream) {
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  int rc = check_params(params);
  if (rc) return rc;
  if (n < 4 || n > 4096) return fail(SWIFT_E_INVAL, "n must be in [4, 4096] (got %d)", n);
  if (batch < 0) return fail(SWIFT_E_INVAL, "batch < 0");
  if (batch == 0) return ok();
  if (!surfaces || !out) return fail(SWIFT_E_INVAL, "surfaces/out is NULL");
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(SWIFT_E_HIP, "cannot select device %d", ctx->device);
  if (2 * params->snr_exclude_r + 1 > n) return fail(SWIFT_E_INVAL, "snr_exclude_r box wider than the surface");
  hipError_t e = launch_snr(surfaces, n, batch, params->snr_exclude_r, out, stream);
  if (e != hipSuccess) return hip_fail(e, "snr launch");
  return ok();
}

int swift_refine_update(swift_ctx* ctx, int32_t P, const swift_match* recs, const float* jac, float* theta,
                        int32_t mode, float max_step, float* step_out, hipStream_t stream) {
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  if (P < 0) return fail(SWIFT_E_INVAL, "P < 0");
  if (P == 0) return ok();
  if (!recs || !theta) return fail(SWIFT_E_INVAL, "recs/theta is NULL");
  if (mode != SWIFT_REFINE_CENTROID && mode != SWIFT_REFINE_NEWTON) return fail(SWIFT_E_INVAL, "bad mode %d", mode);
  if (mode == SWIFT_REFINE_NEWTON && !jac) return fail(SWIFT_E_INVAL, "Newton steps need jac");
  if (!(max_step > 0.0f)) return fail(SWIFT_E_INVAL, "max_step must be > 0");
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(SWIFT_E_HIP, "cannot select device %d", ctx->device);
  hipError_t e = launch_refine(P, recs, jac, theta, mode, max_step, step_out, stream);
  if (e != hipSuccess) return hip_fail(e, "refine launch");
  return ok();
}

int swift_render(swift_ctx* ctx, const uint8_t* src, int32_t S, int32_t src_h, int32_t src_w, int64_t src_pitch,
                 int64_t src_stride, const double* aff, int32_t level, uint8_t* dst, int32_t dst_h, int32_t dst_w,
                 int64_t dst_pitch, int64_t dst_stride, hipStream_t stream) {
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  if (!src || !dst || !aff) return fail(SWIFT_E_INVAL, "src/dst/aff is NULL");
  if (S < 1 || src_h < 1 || src_w < 1 || dst_h < 1 || dst_w < 1) return fail(SWIFT_E_INVAL, "bad sizes");
  if (dst_h > 65535 || S > 65535) return fail(SWIFT_E_INVAL, "dst_h and S must be at most 65535");
  if (level < 0 || level > 12) return fail(SWIFT_E_INVAL, "level must be in [0, 12] (got %d)", level);
  if (src_pitch < src_w || dst_pitch < dst_w) return fail(SWIFT_E_INVAL, "pitch smaller than width");
  if (src_stride < src_pitch * src_h || dst_stride < dst_pitch * dst_h)
    return fail(SWIFT_E_INVAL, "section stride smaller than height * pitch");
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(SWIFT_E_HIP, "cannot select device %d", ctx->device);
  hipError_t e = launch_render(src, src_pitch, src_stride, S, src_h, src_w, aff, level, dst, dst_pitch, dst_stride,
                               dst_h, dst_w, stream, ctx->kt());
  if (e != hipSuccess) return hip_fail(e, "render launch");
  return ok();
}

int swift_stack_windows(swift_ctx* ctx, int32_t S, const double* aff, int32_t level, int32_t grid, int32_t h_l,
                        int32_t w_l, int32_t img_a0, int32_t img_b0, float* theta_a, float* theta_b, int32_t* img_a,
                        int32_t* img_b, hipStream_t stream) {
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  if (!aff || !theta_a || !theta_b || !img_a || !img_b) return fail(SWIFT_E_INVAL, "NULL output or affine");
  if (S < 1 || grid < 1 || h_l < grid || w_l < grid) return fail(SWIFT_E_INVAL, "bad sizes");
  if ((long long)S * grid * grid > (1LL << 30)) return fail(SWIFT_E_INVAL, "too many windows");
  if (level < 0 || level > 12) return fail(SWIFT_E_INVAL, "level must be in [0, 12] (got %d)", level);
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(SWIFT_E_HIP, "cannot select device %d", ctx->device);
  hipError_t e = launch_stack_windows(S, aff, level, grid, h_l, w_l, img_a0, img_b0, theta_a, theta_b, img_a, img_b,
                                      false, stream);
  if (e != hipSuccess) return hip_fail(e, "window launch");
  return ok();
}

// A mesh needs two nodes per axis and a frame of at least one pixel per node;
// the kernels' cell search assumes frame coordinates below 2^16.
static int check_mesh(int grid, int h_l, int w_l) {
  if (grid < 2 || grid > 1024) return fail(SWIFT_E_INVAL, "mesh grid must be in [2, 1024] (got %d)", grid);
  if (h_l < grid || w_l < grid) return fail(SWIFT_E_INVAL, "mesh frame %d x %d smaller than grid %d", h_l, w_l, grid);
  if (h_l > 65535 || w_l > 65535) return fail(SWIFT_E_INVAL, "mesh frame %d x %d above 65535", h_l, w_l);
  return SWIFT_OK;
}

int swift_render_mesh(swift_ctx* ctx, const uint8_t* src, int32_t S, int32_t src_h, int32_t src_w,
                      int64_t src_pitch, int64_t src_stride, const double* tri_aff, int32_t grid, int32_t level,
                      uint8_t* dst, int32_t dst_h, int32_t dst_w, int64_t dst_pitch, int64_t dst_stride,
                      hipStream_t stream) {
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  if (!src || !dst || !tri_aff) return fail(SWIFT_E_INVAL, "src/dst/tri_aff is NULL");
  if (S < 1 || src_h < 1 || src_w < 1 || dst_h < 1 || dst_w < 1) return fail(SWIFT_E_INVAL, "bad sizes");
  if (dst_h > 65535 || S > 65535) return fail(SWIFT_E_INVAL, "dst_h and S must be at most 65535");
  if (level < 0 || level > 12) return fail(SWIFT_E_INVAL, "level must be in [0, 12] (got %d)", level);
  if (src_pitch < src_w || dst_pitch < dst_w) return fail(SWIFT_E_INVAL, "pitch smaller than width");
  if (src_stride < src_pitch * src_h || dst_stride < dst_pitch * dst_h)
    return fail(SWIFT_E_INVAL, "section stride smaller than height * pitch");
  if (check_mesh(grid, dst_h, dst_w) != SWIFT_OK) return SWIFT_E_INVAL;
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(SWIFT_E_HIP, "cannot select device %d", ctx->device);
  hipError_t e = launch_render_mesh(src, src_pitch, src_stride, S, src_h, src_w, tri_aff, grid, level, dst,
                                    dst_pitch, dst_stride, dst_h, dst_w, stream, ctx->kt());
  if (e != hipSuccess) return hip_fail(e, "mesh render launch");
  return ok();
}

int swift_mesh_windows(swift_ctx* ctx, int32_t S, const double* tri_aff, int32_t level, int32_t grid, int32_t h_l,
                       int32_t w_l, int32_t img_a0, int32_t img_b0, float* theta_a, float* theta_b, int32_t* img_a,
                       int32_t* img_b, hipStream_t stream) {
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  if (!tri_aff || !theta_a || !theta_b || !img_a || !img_b) return fail(SWIFT_E_INVAL, "NULL output or affine");
  if (S < 1) return fail(SWIFT_E_INVAL, "bad sizes");
  if (check_mesh(grid, h_l, w_l) != SWIFT_OK) return SWIFT_E_INVAL;
  if ((long long)S * grid * grid > (1LL << 30)) return fail(SWIFT_E_INVAL, "too many windows");
  if (level < 0 || level > 12) return fail(SWIFT_E_INVAL, "level must be in [0, 12] (got %d)", level);
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(SWIFT_E_HIP, "cannot select device %d", ctx->device);
  hipError_t e = launch_stack_windows(S, tri_aff, level, grid, h_l, w_l, img_a0, img_b0, theta_a, theta_b, img_a,
                                      img_b, true, stream);
  if (e != hipSuccess) return hip_fail(e, "mesh window launch");
  return ok();
}

int swift_fit_mesh(swift_ctx* ctx, int32_t S, int32_t grid, const float* theta_a, const float* theta_b,
                   const swift_match* recs, int32_t level, float min_snr, const double* aff, double* tri_aff,
                   int32_t* status, hipStream_t stream) {
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  if (!theta_a || !theta_b || !recs || !aff || !tri_aff) return fail(SWIFT_E_INVAL, "NULL input or affine");
  if (S < 1 || S > 65535) return fail(SWIFT_E_INVAL, "S must be in [1, 65535] (got %d)", S);
  if (grid < 2 || grid > 1024) return fail(SWIFT_E_INVAL, "mesh grid must be in [2, 1024] (got %d)", grid);
  if (level < 0 || level > 12) return fail(SWIFT_E_INVAL, "level must be in [0, 12] (got %d)", level);
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(SWIFT_E_HIP, "cannot select device %d", ctx->device);
  hipError_t e = launch_fit_mesh(S, grid, theta_a, theta_b, recs, level, min_snr, aff, tri_aff, status, stream,
                                 ctx->kt());
  if (e != hipSuccess) return hip_fail(e, "mesh fit launch");
  return ok();
}

int swift_fit_sections(swift_ctx* ctx, int32_t S, int32_t per_section, const float* theta_a, const float* theta_b,
                       const swift_match* recs, int32_t level, float min_snr, double* aff, int32_t* status,
                       hipStream_t stream) {
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  if (!theta_a || !theta_b || !recs || !aff) return fail(SWIFT_E_INVAL, "NULL input or affine");
  if (S < 1 || per_section < 1) return fail(SWIFT_E_INVAL, "bad sizes");
  if (level < 0 || level > 12) return fail(SWIFT_E_INVAL, "level must be in [0, 12] (got %d)", level);
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(SWIFT_E_HIP, "cannot select device %d", ctx->device);
  hipError_t e = launch_fit_sections(S, per_section, theta_a, theta_b, recs, level, min_snr, aff, status, stream);
  if (e != hipSuccess) return hip_fail(e, "fit launch");
  return ok();
}

static int size_index(int n) {
  for (int i = 0; i < SWIFT_NSIZES; ++i)
    if (kSizes[i] == n) return i;
  return -1;
}

int swift_plan(swift_ctx* ctx, int32_t n, int32_t fwd_variant, int32_t inv_variant, int32_t chunks,
               int32_t* fwd_rows, int32_t* inv_rows, int32_t* chunks_out) {
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  const int i = size_index(n);
  if (i < 0) return fail(SWIFT_E_INVAL, "n must be one of 64, 128, 256, 512, 1024 (got %d)", n);
  if (fwd_variant > 1 || inv_variant > 1) {
    if (!(fwd_variant == kFusedVariant && n <= kFusedMaxN && inv_variant <= 1))
      return fail(SWIFT_E_INVAL, "variants are 0, 1 or -1 (keep), and forward variant 2 (one workgroup per pair) "
                                 "for n <= %d", kFusedMaxN);
  }
  if (chunks >= 0 && !valid_chunks(chunks)) return fail(SWIFT_E_INVAL, "chunks are 1, 2, 4, 8 or -1 (keep)");
  if (fwd_variant >= 0) ctx->alt_fwd[i] = (uint8_t)fwd_variant;
  if (inv_variant >= 0) ctx->alt_inv[i] = (uint8_t)inv_variant;
  if (chunks >= 0) ctx->chunks[i] = (uint8_t)chunks;
  const bool fused = ctx->alt_fwd[i] == kFusedVariant;
  if (fwd_rows) *fwd_rows = fused ? n : n / fwd_blocks_n(n, ctx->alt_fwd[i] == 1);
  if (inv_rows) *inv_rows = fused ? n : n / inv_blocks_n(n, ctx->alt_inv[i] != 0);
  if (chunks_out) *chunks_out = ctx->chunks[i];
  return ok();
}

// Synthetic tuning input: a uint8 image of hashed noise.
__global__ void k_tune_image(uint8_t* img, int64_t n_px) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n_px) return;
  uint32_t h = (uint32_t)i * 2654435761u;
  h ^= h >> 15;
  h *= 2246822519u;
  h ^= h >> 13;
  img[i] = (uint8_t)(h >> 24);
}

namespace {
// Device buffers of one tuning batch, freed on scope exit.
struct TuneBufs {
  void* p[6] = {};
  ~TuneBufs() {
    for (void* q : p)
      if (q) (void)hipFree(q);
  }
};
}  // namespace

int swift_autotune(swift_ctx* ctx, const int32_t* sizes, int32_t n_sizes, int32_t pairs_per_size,
                   float* times_ms) {
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  if (n_sizes < 0 || (n_sizes > 0 && !sizes)) return fail(SWIFT_E_INVAL, "bad size list");
  for (int k = 0; k < n_sizes; ++k)
    if (size_index(sizes[k]) < 0) return fail(SWIFT_E_INVAL, "unsupported window size %d", sizes[k]);
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(SWIFT_E_HIP, "cannot select device %d", ctx->device);
  hipStream_t st = ctx->gs[0];
  bool tuned[SWIFT_NSIZES] = {};
  for (int k = 0; k < n_sizes; ++k) {
    const int n = sizes[k], si = size_index(n);
    // square grid of windows on one image, capped at 1 GiB of pixels
    int P = pairs_per_size > 0 ? pairs_per_size : 512;
    int grid = (int)ceil(sqrt((double)P));
    while (grid > 1 && (double)(grid + 2) * n * (grid + 2) * n > (double)(1u << 30)) --grid;
    P = min(P, grid * grid);
    const int side = (grid + 2) * n;
    TuneBufs b;
    hipError_t e = hipMalloc(&b.p[0], (size_t)side * side);
    const size_t npairs = (size_t)P;
    if (e == hipSuccess) e = hipMalloc(&b.p[1], sizeof(swift_image));
    if (e == hipSuccess) e = hipMalloc(&b.p[2], 2 * npairs * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&b.p[3], 2 * npairs * 8 * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&b.p[4], npairs * sizeof(swift_match));
    if (e != hipSuccess) return hip_fail(e, "autotune buffers");
    const int64_t npx = (int64_t)side * side;
    k_tune_image<<<(unsigned)((npx + 255) / 256), 256, 0, st>>>((uint8_t*)b.p[0], npx);
    swift_image im;
    memset(&im, 0, sizeof(im));
    im.data = b.p[0];
    im.width = side;
    im.height = side;
    im.pitch = side;
    im.dtype = SWIFT_U8;
    std::vector<int32_t> idx(2 * npairs, 0);
    std::vector<float> th(2 * npairs * 8);
    for (size_t q = 0; q < npairs; ++q) {
      const float cx = (float)((q % grid) + 1) * n + n / 2, cy = (float)((q / grid) + 1) * n + n / 2;
      const float a[8] = {cx, cy, 1, 0, 0.3f, 0, 1, -0.2f};
      const float bb[8] = {cx, cy, 1, 0, -0.1f, 0, 1, 0.4f};
      for (int j = 0; j < 8; ++j) {
        th[q * 8 + j] = a[j];
        th[(npairs + q) * 8 + j] = bb[j];
      }
    }
    e = hipMemcpyAsync(b.p[1], &im, sizeof(im), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(b.p[2], idx.data(), idx.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(b.p[3], th.data(), th.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "autotune inputs");
    swift_pairs pr;
    memset(&pr, 0, sizeof(pr));
    pr.n_pairs = P;
    pr.size_count[si] = P;
    pr.img_a = (const int32_t*)b.p[2];
    pr.img_b = (const int32_t*)b.p[2] + npairs;
    pr.theta_a = (const float*)b.p[3];
    pr.theta_b = (const float*)b.p[3] + npairs * 8;
    swift_params prm;
    memset(&prm, 0, sizeof(prm));
    prm.p = 0.65f;
    prm.eps_rel = 1e-4f;
    prm.taper_frac = 0.25f;
    prm.centroid_r = 1;
    const Layout L = make_layout(&pr);
    e = hipMalloc(&b.p[5], L.total);
    if (e != hipSuccess) return hip_fail(e, "autotune workspace");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      if (e0) (void)hipEventDestroy(e0);
      return fail(SWIFT_E_HIP, "autotune events");
    }
    const uint8_t keep_f = ctx->alt_fwd[si], keep_i = ctx->alt_inv[si], keep_c = ctx->chunks[si];
    int rc = SWIFT_OK;
    // slots 0..3: the row variants in one chunk; 4..6: the best of them in
    // 2, 4, 8 chunks on two streams; 7 (n <= kFusedMaxN): one workgroup per
    // pair.  vv: bit 0 the alternative forward rows, bit 1 the alternative
    // inverse rows, 4 the one-workgroup kernel.  Each slot is timed as the
    // mean of 3 batches, in kTuneRounds rounds that visit the slots in turn
    // (so slow drifts of the clock touch every slot alike), and keeps its
    // fastest round.  A slot replaces the current choice only when it is at
    // least kTuneMargin faster: differences within the run-to-run spread do
    // not move the plan off the defaults.
    float tmin[kTuneSlots];
    for (int v = 0; v < kTuneSlots; ++v) tmin[v] = -1.0f;
    int best_v = 0, best_c = 1;
    auto slot_cfg = [&](int v, int& af, bool& ai, int& ch, int& vv) {
      vv = v < 4 ? v : v == 7 ? 4 : best_v;
      ch = v < 4 || v == 7 ? 1 : (v == 4 ? 2 : v == 5 ? 4 : 8);
      af = vv == 4 ? kFusedVariant : (vv & 1);
      ai = vv != 4 && (vv & 2) != 0;
      return ch <= P && (af != 1 || fwd_blocks_n(n, true) != fwd_blocks_n(n, false)) &&
             (!ai || inv_blocks_n(n, true) != inv_blocks_n(n, false)) && (vv != 4 || n <= kFusedMaxN) &&
             !(v >= 4 && v < 7 && best_v == 4);
    };
    auto time_slot = [&](int v, bool warm) {
      int af, ch, vv;
      bool ai;
      if (!slot_cfg(v, af, ai, ch, vv)) return;
      ctx->alt_fwd[si] = (uint8_t)af;
      ctx->alt_inv[si] = ai;
      ctx->chunks[si] = (uint8_t)ch;
      float ms = -1.0f;
      if (warm)
        rc = enqueue_match(ctx, (const swift_image*)b.p[1], 1, &pr, &prm, (swift_match*)b.p[4], nullptr, nullptr,
                           b.p[5], st, false, nullptr);
      if (rc == SWIFT_OK) rc = hipEventRecord(e0, st) == hipSuccess ? SWIFT_OK : fail(SWIFT_E_HIP, "event");
      for (int r = 0; r < 3 && rc == SWIFT_OK; ++r)
        rc = enqueue_match(ctx, (const swift_image*)b.p[1], 1, &pr, &prm, (swift_match*)b.p[4], nullptr, nullptr,
                           b.p[5], st, false, nullptr);
      if (rc == SWIFT_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = fail(SWIFT_E_HIP, "autotune timing");
      if (rc == SWIFT_OK) {
        ms /= 3.0f;
        tmin[v] = tmin[v] < 0.0f ? ms : fminf(tmin[v], ms);
      }
    };
    // the row variants and the one-workgroup kernel, then the chunk counts of
    // the winner
    const int phase_a[5] = {0, 1, 2, 3, 7}, phase_b[3] = {4, 5, 6};
    for (int r = 0; r < kTuneRounds && rc == SWIFT_OK; ++r)
      for (int i = 0; i < 5 && rc == SWIFT_OK; ++i) time_slot(phase_a[i], r == 0);
    float best = tmin[0];
    for (int i = 1; i < 5 && rc == SWIFT_OK; ++i) {
      const int v = phase_a[i];
      if (tmin[v] > 0.0f && tmin[v] < best * (1.0f - kTuneMargin)) {
        best = tmin[v];
        best_v = v < 4 ? v : 4;
      }
    }
    for (int r = 0; r < kTuneRounds && rc == SWIFT_OK; ++r)
      for (int i = 0; i < 3 && rc == SWIFT_OK; ++i) time_slot(phase_b[i], r == 0);
    const float row_best = best;
    for (int i = 0; i < 3 && rc == SWIFT_OK; ++i) {
      const int v = phase_b[i];
      if (tmin[v] > 0.0f && tmin[v] < row_best * (1.0f - kTuneMargin) && tmin[v] < best) {
        best = tmin[v];
        best_c = v == 4 ? 2 : v == 5 ? 4 : 8;
      }
    }
    if (times_ms)
      for (int v = 0; v < kTuneSlots; ++v) times_ms[k * kTuneSlots + v] = tmin[v];
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != SWIFT_OK) {
      ctx->alt_fwd[si] = keep_f;
      ctx->alt_inv[si] = keep_i;
      ctx->chunks[si] = keep_c;
      return rc;
    }
    ctx->alt_fwd[si] = best_v == 4 ? kFusedVariant : (best_v & 1);
    ctx->alt_inv[si] = best_v != 4 && (best_v & 2) != 0;
    ctx->chunks[si] = (uint8_t)best_c;
    tuned[si] = true;
  }
  if (!ctx->tune_path.empty() && n_sizes > 0 && !tune_cache_store(ctx, tuned))
    return fail(SWIFT_E_INVAL, "plan tuned but the tune cache %s could not be written", ctx->tune_path.c_str());
  return ok();
}

int swift_profile_enable(swift_ctx* ctx, int enable) {
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  ctx->profile = enable != 0;
  return ok();
}

int swift_profile_read(swift_ctx* ctx, int32_t max_kernels, char* names, int32_t* launches, double* total_ms,
                       int32_t* n_kernels) {
  if (!ctx) return fail(SWIFT_E_INVAL, "ctx is NULL");
  if (!n_kernels || max_kernels < 0 || (max_kernels > 0 && (!names || !launches || !total_ms)))
    return fail(SWIFT_E_INVAL, "bad output arrays");
  DeviceGuard dg(ctx->device);
  std::map<std::string, std::pair<int, double>> agg;
  EventTimer& t = ctx->timer;
  int rc = SWIFT_OK;
  for (auto& r : t.recs) {
    float ms = 0.0f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) rc = hip_fail(e, "hipEventElapsedTime");
    auto& v = agg[r.name];
    v.first += 1;
    v.second += ms;
    t.pool.push_back(r.a);
    t.pool.push_back(r.b);
  }
  t.recs.clear();
  if (t.failed) rc = fail(SWIFT_E_HIP, "event record failed while profiling");
  t.failed = false;
  int i = 0;
  for (auto& kv : agg) {
    if (i < max_kernels) {
      snprintf(names + 64 * i, 64, "%s", kv.first.c_str());
      launches[i] = kv.second.first;
      total_ms[i] = kv.second.second;
    }
    ++i;
  }
  *n_kernels = i;
  return rc ? rc : ok();
}

}  // extern "C"
