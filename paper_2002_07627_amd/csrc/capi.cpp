// Host runtime and C interface of the IMF library (include/imf.h).
//
// One request runs Algorithm 1 of Sec. 2.1.5 on the device:
//   rasterize the oriented tools (cached per tool and direction),
//   forward transform of rho_O once, then per batch of orientations: tool
//   spectra (cached or regenerated), fused product + inverse transform over the
//   query box, exact rounding / guard-band recheck, sharp-point minimum with
//   the running minimum and the masks; finally F_max, fbar, B and Gamma.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <cstdarg>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <unordered_map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/imf.h"
#include "imf_internal.h"

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err = "no error";

static imf_status fail(imf_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static imf_status fail(imf_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(call)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(e_ == hipErrorOutOfMemory ? IMF_ENOMEM : IMF_EDEVICE, "%s: %s (%s:%d)", \
                  #call, hipGetErrorString(e_), __FILE__, __LINE__);                    \
  } while (0)

#define STCHK(call)                    \
  do {                                 \
    imf_status s_ = (call);            \
    if (s_ != IMF_OK) return s_;       \
  } while (0)

extern "C" const char* imf_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// FFT sizes: 2^a 3^b 5^c 7^d with a >= 1, up to 1024
// ---------------------------------------------------------------------------
static imf_fft_len make_len(int n) {
  imf_fft_len L{};
  L.n = n;
  int m = n;
  auto push = [&](int r) { L.radix[L.nstages++] = r; m /= r; };
  while (m % 8 == 0 && L.nstages < 8) push(8);
  while (m % 4 == 0 && L.nstages < 8) push(4);
  while (m % 2 == 0 && L.nstages < 8) push(2);
  while (m % 3 == 0 && L.nstages < 8) push(3);
  while (m % 5 == 0 && L.nstages < 8) push(5);
  while (m % 7 == 0 && L.nstages < 8) push(7);
  if (m != 1) {
    L.nstages = -1;
    return L;
  }
  int ns = 1;
  for (int s = 0; s < L.nstages; s++) {
    L.Ns[s] = ns;
    L.invNs[s] = 1.0f / (float)ns;
    L.step[s] = n / (ns * L.radix[s]);
    ns *= L.radix[s];
  }
  return L;
}

static bool smooth(int n) {
  if (n < 2 || n % 2) return false;
  int m = n;
  for (int p : {2, 3, 5, 7})
    while (m % p == 0) m /= p;
  return m == 1;
}

extern "C" int imf_fft_size(int n) {
  if (n <= 1) return 1;
  // lengths with compile-time transform kernels, when within 25% of n
  static const int fast[] = {64, 96, 128, 160, 192, 216, 224, 256, 288, 320,
                             384, 448, 512, 576, 640, 768, 1024};
  for (int m : fast)
    if (m >= n) {
      if (m <= n + n / 4) return m;
      break;
    }
  // cheapest smooth length in [n, 1.3 n]: cost n log n with a surcharge for
  // the slower radix-5/7 stages
  double best = 1e300;
  int pick = -1;
  for (int m = std::max(n, 2); m <= 1024 && m <= (int)(1.3 * n) + 2; m++) {
    if (!smooth(m)) continue;
    imf_fft_len L = make_len(m);
    if (L.nstages < 0) continue;
    int slow = 0;
    for (int s = 0; s < L.nstages; s++) slow += (L.radix[s] == 5 || L.radix[s] == 7);
    const double c = m * std::log2((double)m) * (1.0 + 0.15 * slow) * (1.0 + 0.02 * L.nstages);
    if (c < best) {
      best = c;
      pick = m;
    }
  }
  return pick;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct OrientEntry {
  int ext[IMF_EXT_INTS];
  int s_axis;       // 0..2: sharp-point runs along that axis; 3: along sv
  int sv[3];        // lattice vector of the sharp-point runs
  int maxlen;       // longest sharp-point run
  int n_pow2;       // the first n_pow2 sharp-point runs have power-of-two lengths
  unsigned lvl_used;  // bit s-1: some sharp-point run reads sparse-table level s
  const imf_run* truns;
  const imf_run* sruns;
  const imf_run* sxruns;
};

struct SpecEntry {
  float2* ptr;
  size_t bytes;
  uint64_t tick;
  hipEvent_t ready;  // recorded after the spectrum is written
};

struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  unsigned int* host = nullptr;  // pinned: counters copied back at the end
  // A serving worker's arena is used by its own stream only, and that stream
  // is idle between requests: when it grows, the old buffer is retired to the
  // context instead of freed (a free waits for the whole device, every other
  // worker's requests included).
  bool worker = false;
};

struct Request;  // serving

struct imf_ctx {
  int device = 0;
  size_t budget = 0;
  size_t spec_bytes = 0, arena_bytes = 0, raster_bytes = 0;
  std::recursive_mutex mu;
  std::vector<imf_tool> tools;
  struct VoxTool {
    uint8_t* dev = nullptr;  // labels on the device (voxel-model tools only)
    int dim[3] = {0, 0, 0}, org[3] = {0, 0, 0};
  };
  std::vector<VoxTool> vtools;  // parallel to tools
  std::map<std::string, OrientEntry> rasters;
  std::vector<void*> raster_pools;
  std::map<std::string, SpecEntry> spectra;
  std::map<int, float2*> twiddles;
  // autotuned launch parameters per request shape (method, grid, transform sizes)
  struct Tuned {
    int batch = 8;     // orientations per batch
    int shape = -1;    // block shape of the sharp-point minimum (-1: context default)
    int wg = 0;        // resident workgroups per CU of its list pass (0: context default)
    int fft = 0;       // transform plans of the inverse z, y, x passes (2 bits each)
  };
  std::map<std::string, Tuned> tuned;
  int force_shape = -1, force_wg = 0;  // set while the autotuner times a candidate
  int force_fft = -1;
  uint64_t tick = 0;
  Arena arena;
  // retired worker arenas: used by nobody, freed (one device synchronization
  // for all) when a reservation needs their room, and at the end
  std::vector<char*> retired;
  size_t retired_bytes = 0;
  hipStream_t internal = nullptr;
  // serving
  std::mutex smu;
  std::condition_variable scv;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<uint64_t, std::shared_ptr<Request>> reqs;
  std::vector<std::thread> workers;
  bool stop = false;
  uint64_t next_ticket = 1;
  size_t inflight_bytes = 0;
  // requests run at once by the serving loop, each on its own stream.  Two:
  // with four, requests whose streams shared a hardware queue with a long
  // request's stream waited behind its kernels (10-25 times their time
  // alone on the 64-request mix at 0.7 load, p99 546 ms); with two, p50 29
  // ms and p99 206 ms against 168 ms for the largest request alone
  int max_inflight = 2;
  int n_running = 0;
  // captured requests: signature -> instantiated graph and the host-side
  // statistics of its launch sequence (the context lock guards both maps)
  struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    double kbytes[16], kops[16];
    std::vector<double> mf_ops, mf_bytes;
    int kept_at = -1;
    uint64_t tick = 0;
  };
  std::unordered_map<std::string, GraphEntry> graphs;
  std::unordered_map<std::string, int> graph_seen;
  uint64_t graph_tick = 0;
  hipStream_t capture = nullptr;  // private stream graphs are captured on
  unsigned int* couple_scratch = nullptr;  // device word for the coupling reductions
  int mf_shape = 2;  // wave block shape of the sharp-point minimum (imf_block_dims)
  int n_cu = 256;     // compute units of the device
  int mf_wg_per_cu = 8;  // resident workgroups per CU of the sharp-point minimum (list pass)
  // grids below this many voxels skip the branch and bound: its three short
  // launches per orientation cost more than the blocks they save
  long long bound_min_voxels = 1000000;
  // sharp-point runs along lattice vectors where they are fewer (3D)
  bool lattice_runs = true;
  // process orientations in farthest-point order of their tool axes
  bool spread_order = true;
  // list pass: the waves of a workgroup (consecutive kept blocks, mostly x
  // neighbours) gather the same runs in step, so they share L1 lines:
  // 0 off, 1 four waves, 2 eight waves per workgroup
  int mf_sync = 2;
  // density requests at lambda F_max keep the overlaps of every orientation
  // when they fit (otherwise a second pass decides the band)
  bool overlap_stack = true;
  // the exact F_max of the last density request at lambda F_max of each
  // request shape (grid, tools, orientations, fixtures; not the design), and
  // the relative width of the bracket listed around lambda times it next time
  struct Hint {
    unsigned long long F[3] = {0, 0, 0};  // the last three exact maxima, newest first (0: none)
    double delta = 0;                     // relative half-width of the next bracket
    double listed = 0;                    // bracket entries per orientation last time
  };
  std::map<std::string, Hint> hints;
  // fraction of (block, orientation) pairs the bound kept in the last request
  // with a gamma stack of each shape: sizes the next compact stack
  std::map<std::string, double> gkept;
  bool use_hints = true;
  // the inverse x pass's appends: -1 deferred after a long bracket, 0 never
  // deferred, 1 always (IMF_DEFER_APPENDS)
  int defer_mode = -1;
  // gamma stack of the kept blocks only, at this fraction of all blocks for
  // a request shape not seen before (0: always the full stack), used when
  // the full stack would take more than 1/16 of the budget (room for cached
  // spectra) or always when set from the environment
  double compact_gamma = 0.5;
  bool compact_forced = false;
};

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static imf_status arena_free_retired(imf_ctx* c) {
  if (c->retired.empty()) return IMF_OK;
  HIPCHK(hipDeviceSynchronize());
  for (char* b : c->retired) HIPCHK(hipFree(b));
  c->retired.clear();
  c->arena_bytes -= c->retired_bytes;
  c->retired_bytes = 0;
  return IMF_OK;
}

// Free cached tool spectra, least recently used first, until `need` bytes
// are free.  Called under the context lock before the request being planned
// takes its spectrum slots: after one device synchronization no launched
// request reads a spectrum, and none can be launched meanwhile; captured
// graphs, which hold spectrum addresses, are dropped.
static imf_status evict_spectra(imf_ctx* c, size_t need) {
  if (c->spectra.empty() || need == 0) return IMF_OK;
  HIPCHK(hipDeviceSynchronize());
  std::vector<std::pair<uint64_t, std::string>> order;
  order.reserve(c->spectra.size());
  for (const auto& kv : c->spectra) order.emplace_back(kv.second.tick, kv.first);
  std::sort(order.begin(), order.end());
  size_t freed = 0;
  for (const auto& o : order) {
    if (freed >= need) break;
    auto it = c->spectra.find(o.second);
    HIPCHK(hipFree(it->second.ptr));
    if (it->second.ready) hipEventDestroy(it->second.ready);
    c->spec_bytes -= it->second.bytes;
    freed += it->second.bytes;
    c->spectra.erase(it);
  }
  for (auto& kv : c->graphs)
    if (kv.second.exec) hipGraphExecDestroy(kv.second.exec);
  c->graphs.clear();
  c->graph_seen.clear();
  return IMF_OK;
}

static imf_status arena_reserve(imf_ctx* c, Arena& a, size_t bytes) {
  if (!a.host) HIPCHK(hipHostMalloc((void**)&a.host, 1 << 16, hipHostMallocDefault));
  if (a.cap >= bytes) {
    a.used = 0;
    return IMF_OK;
  }
  if (a.base && a.worker) {
    c->retired.push_back(a.base);
    c->retired_bytes += a.cap;
    a.base = nullptr;
    a.cap = 0;
  } else if (a.base) {
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipFree(a.base));
    c->arena_bytes -= a.cap;
    a.base = nullptr;
    a.cap = 0;
  }
  if (c->spec_bytes + c->arena_bytes + c->raster_bytes + bytes > c->budget)
    STCHK(arena_free_retired(c));
  // a workspace comes before cached spectra
  if (c->spec_bytes + c->arena_bytes + c->raster_bytes + bytes > c->budget)
    STCHK(evict_spectra(c, c->spec_bytes + c->arena_bytes + c->raster_bytes + bytes - c->budget));
  const size_t others = c->spec_bytes + c->arena_bytes + c->raster_bytes;
  if (others + bytes > c->budget)
    return fail(IMF_ENOMEM, "workspace of %zu bytes exceeds the context budget (%zu used of %zu)",
                bytes, others, c->budget);
  HIPCHK(hipMalloc(&a.base, bytes));
  a.cap = bytes;
  a.used = 0;
  c->arena_bytes += bytes;
  return IMF_OK;
}

template <class T>
static T* carve(Arena& a, size_t count) {
  T* p = (T*)(a.base + a.used);
  a.used += align256(count * sizeof(T));
  return p;
}

static imf_status get_twiddles(imf_ctx* c, int n, const float2** out) {
  auto it = c->twiddles.find(n);
  if (it != c->twiddles.end()) {
    *out = it->second;
    return IMF_OK;
  }
  float2* p = nullptr;
  HIPCHK(hipMalloc(&p, sizeof(float2) * std::max(n, 1)));
  HIPCHK(imf_launch_twiddles(p, n, c->internal));
  HIPCHK(hipStreamSynchronize(c->internal));
  c->twiddles[n] = p;
  *out = p;
  return IMF_OK;
}

extern "C" imf_status imf_create(int device, size_t hbm_budget_bytes, imf_ctx** ctx) {
  if (!ctx) return fail(IMF_EINVAL, "ctx is NULL");
  int n = 0;
  HIPCHK(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(IMF_EINVAL, "device %d of %d", device, n);
  HIPCHK(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(IMF_EDEVICE, "device %d is %s; this library is built for gfx950", device,
                prop.gcnArchName);
  size_t fr = 0, tot = 0;
  HIPCHK(hipMemGetInfo(&fr, &tot));
  // the allocation-free planner's scratch: its device address on this device
  {
    const hipError_t e = imf_plan_scratch_init(device);
    if (e != hipSuccess)
      return fail(IMF_EDEVICE, "planner scratch address: %s", hipGetErrorString(e));
  }
  imf_ctx* c = new imf_ctx();
  c->device = device;
  c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)fr);
  if (const char* e = std::getenv("IMF_MINFILTER_SHAPE"))
    c->mf_shape = std::max(0, std::min(4, std::atoi(e)));
  c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  if (const char* e = std::getenv("IMF_BOUND_MIN_VOXELS")) c->bound_min_voxels = std::atoll(e);
  if (const char* e = std::getenv("IMF_AXIS_RUNS")) c->lattice_runs = std::atoi(e) == 0;
  if (const char* e = std::getenv("IMF_GIVEN_ORDER")) c->spread_order = std::atoi(e) == 0;
  if (const char* e = std::getenv("IMF_MINFILTER_SYNC")) c->mf_sync = std::atoi(e);
  if (const char* e = std::getenv("IMF_OVERLAP_STACK")) c->overlap_stack = std::atoi(e) != 0;
  if (const char* e = std::getenv("IMF_THRESHOLD_HINTS")) c->use_hints = std::atoi(e) != 0;
  if (const char* e = std::getenv("IMF_DEFER_APPENDS")) c->defer_mode = std::atoi(e) != 0;
  if (const char* e = std::getenv("IMF_COMPACT_GAMMA")) {
    c->compact_gamma = std::max(0.0, std::min(1.0, std::atof(e)));
    c->compact_forced = true;
  }
  if (const char* e = std::getenv("IMF_SERVE_WORKERS"))
    c->max_inflight = std::max(1, std::min(16, std::atoi(e)));
  if (const char* e = std::getenv("IMF_MINFILTER_WG_PER_CU"))
    c->mf_wg_per_cu = std::max(1, std::min(16, std::atoi(e)));
  if (hipStreamCreateWithFlags(&c->internal, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return fail(IMF_EDEVICE, "stream creation failed");
  }
  *ctx = c;
  return IMF_OK;
}

static void serve_shutdown(imf_ctx* c);

extern "C" imf_status imf_destroy(imf_ctx* c) {
  if (!c) return IMF_OK;
  serve_shutdown(c);
  hipSetDevice(c->device);
  hipDeviceSynchronize();
  for (auto& kv : c->spectra) {
    hipFree(kv.second.ptr);
    if (kv.second.ready) hipEventDestroy(kv.second.ready);
  }
  if (c->arena.host) hipHostFree(c->arena.host);
  for (void* p : c->raster_pools) hipFree(p);
  for (auto& kv : c->twiddles) hipFree(kv.second);
  if (c->arena.base) hipFree(c->arena.base);
  for (char* b : c->retired) hipFree(b);
  for (auto& kv : c->graphs)
    if (kv.second.exec) hipGraphExecDestroy(kv.second.exec);
  if (c->internal) hipStreamDestroy(c->internal);
  if (c->capture) hipStreamDestroy(c->capture);
  if (c->couple_scratch) hipFree(c->couple_scratch);
  for (auto& v : c->vtools)
    if (v.dev) hipFree(v.dev);
  delete c;
  return IMF_OK;
}

extern "C" imf_status imf_tool_register(imf_ctx* c, const imf_tool* t, int* id) {
  if (!c || !t || !id) return fail(IMF_EINVAL, "NULL argument");
  if (t->kind < 0 || t->kind > 2) return fail(IMF_EINVAL, "unknown tool kind %d", t->kind);
  if (!(t->cutter_r > 0 && t->cutter_len > 0 && t->holder_r >= 0 && t->holder_len >= 0) ||
      !std::isfinite(t->cutter_r + t->cutter_len + t->holder_r + t->holder_len))
    return fail(IMF_EINVAL, "tool sizes must be positive (holder may be empty)");
  if (t->cutter_len + t->holder_len > 400 || t->cutter_r > 200 || t->holder_r > 200)
    return fail(IMF_EINVAL, "tool larger than 400 voxels");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  c->tools.push_back(*t);
  c->vtools.emplace_back();
  *id = (int)c->tools.size() - 1;
  return IMF_OK;
}

extern "C" imf_status imf_tool_register_voxel(imf_ctx* c, int nx, int ny, int nz,
                                              const uint8_t* labels, const int origin[3],
                                              int* id) {
  if (!c || !labels || !origin || !id) return fail(IMF_EINVAL, "NULL argument");
  if (nx < 1 || ny < 1 || nz < 1 || nx > 1024 || ny > 1024 || nz > 1024)
    return fail(IMF_EINVAL, "voxel tool of %d x %d x %d voxels", nx, ny, nz);
  const int dims[3] = {nx, ny, nz};
  for (int a = 0; a < 3; a++)
    if (origin[a] < 0 || origin[a] >= dims[a]) return fail(IMF_EINVAL, "tip outside the labels");
  const size_t n = (size_t)nx * ny * nz;
  bool any_cut = false;
  for (size_t i = 0; i < n; i++) {
    if (labels[i] > 2) return fail(IMF_EINVAL, "labels must be 0, 1 or 2");
    any_cut = any_cut || labels[i] == 2;
  }
  if (!any_cut) return fail(IMF_EINVAL, "a voxel tool needs cutter voxels");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  HIPCHK(hipSetDevice(c->device));
  imf_ctx::VoxTool v;
  HIPCHK(hipMalloc(&v.dev, n));
  if (hipMemcpy(v.dev, labels, n, hipMemcpyHostToDevice) != hipSuccess) {
    hipFree(v.dev);
    return fail(IMF_EDEVICE, "voxel tool upload");
  }
  for (int a = 0; a < 3; a++) {
    v.dim[a] = dims[a];
    v.org[a] = origin[a];
  }
  imf_tool t{};
  t.kind = IMF_TOOL_VOXEL;
  c->tools.push_back(t);
  c->vtools.push_back(v);
  *id = (int)c->tools.size() - 1;
  return IMF_OK;
}

// ---------------------------------------------------------------------------
// orientations of a request
// ---------------------------------------------------------------------------
struct Orient {
  int index;  // position in the request (outputs are indexed by it)
  int tool;
  double d[3];
  long long v[3];
  double R[9];  // rotation (IMF_DIR_ROTATION)
  std::string key;
};

static bool is_half_int(double x) { return std::fabs(x * 2 - std::rint(x * 2)) == 0 && std::fabs(x) < 1e6; }

static imf_status enumerate(imf_ctx* c, const imf_request* r, std::vector<Orient>& out) {
  out.clear();
  const int nd = r->ndim;
  size_t k = 0;
  for (int i = 0; i < r->n_tools; i++) {
    const int tid = r->tool_ids[i];
    if (tid < 0 || tid >= (int)c->tools.size()) return fail(IMF_EINVAL, "unknown tool id %d", tid);
    const imf_tool& t = c->tools[tid];
    if (t.kind == IMF_TOOL_RECT2D && nd != 2)
      return fail(IMF_EINVAL, "RECT2D tools are 2D only");
    if (t.kind == IMF_TOOL_VOXEL && r->dir_kind != IMF_DIR_ROTATION)
      return fail(IMF_EINVAL, "voxel tools need rotation matrices (IMF_DIR_ROTATION)");
    if (r->dir_kind == IMF_DIR_ROTATION && nd != 3)
      return fail(IMF_EINVAL, "rotation matrices are for 3D requests");
    if (r->dir_kind == IMF_DIR_LATTICE &&
        !(is_half_int(t.cutter_r) && is_half_int(t.cutter_len) && is_half_int(t.holder_r) &&
          is_half_int(t.holder_len)))
      return fail(IMF_EINVAL, "lattice directions need tool sizes that are multiples of 1/2");
    if (r->n_dirs[i] < 1) return fail(IMF_EINVAL, "tool %d has no directions", i);
    for (int j = 0; j < r->n_dirs[i]; j++, k++) {
      Orient o{};
      o.tool = tid;
      if (r->dir_kind == IMF_DIR_LATTICE) {
        const int32_t* v = (const int32_t*)r->dirs + k * nd;
        long long n2 = 0;
        for (int a = 0; a < nd; a++) {
          o.v[a] = v[a];
          n2 += (long long)v[a] * v[a];
        }
        if (n2 == 0) return fail(IMF_EINVAL, "direction %zu is zero", k);
        if (n2 > 1000000) return fail(IMF_EINVAL, "lattice direction %zu too long", k);
        for (int a = 0; a < nd; a++) o.d[a] = (double)o.v[a] / std::sqrt((double)n2);
      } else if (r->dir_kind == IMF_DIR_F64) {
        const double* v = (const double*)r->dirs + k * nd;
        double n2 = 0;
        for (int a = 0; a < nd; a++) {
          o.d[a] = v[a];
          n2 += v[a] * v[a];
        }
        if (!(std::fabs(std::sqrt(n2) - 1.0) <= 1e-12))
          return fail(IMF_EINVAL, "direction %zu is not a unit vector", k);
      } else if (r->dir_kind == IMF_DIR_ROTATION) {
        const double* R = (const double*)r->dirs + k * 9;
        for (int i = 0; i < 9; i++) o.R[i] = R[i];
        for (int i = 0; i < 3; i++)
          for (int j = 0; j < 3; j++) {
            const double dot = R[3 * i] * R[3 * j] + R[3 * i + 1] * R[3 * j + 1] +
                               R[3 * i + 2] * R[3 * j + 2];
            if (!(std::fabs(dot - (i == j ? 1.0 : 0.0)) <= 1e-9))
              return fail(IMF_EINVAL, "rotation %zu is not orthonormal", k);
          }
        const double det = R[0] * (R[4] * R[8] - R[5] * R[7]) -
                           R[1] * (R[3] * R[8] - R[5] * R[6]) + R[2] * (R[3] * R[7] - R[4] * R[6]);
        if (!(det > 0)) return fail(IMF_EINVAL, "rotation %zu has determinant -1", k);
        o.d[0] = R[2];  // image of the tool's +z axis
        o.d[1] = R[5];
        o.d[2] = R[8];
      } else {
        return fail(IMF_EINVAL, "unknown dir_kind %d", r->dir_kind);
      }
      char buf[400];
      if (r->dir_kind == IMF_DIR_LATTICE)
        snprintf(buf, sizeof buf, "%d|%d|L|%d|%lld,%lld,%lld", tid, nd, r->sharp, o.v[0], o.v[1],
                 o.v[2]);
      else if (r->dir_kind == IMF_DIR_ROTATION && t.kind == IMF_TOOL_VOXEL)
        snprintf(buf, sizeof buf, "%d|%d|R|%d|%a,%a,%a,%a,%a,%a,%a,%a,%a", tid, nd, r->sharp,
                 o.R[0], o.R[1], o.R[2], o.R[3], o.R[4], o.R[5], o.R[6], o.R[7], o.R[8]);
      else
        snprintf(buf, sizeof buf, "%d|%d|F|%d|%a,%a,%a", tid, nd, r->sharp, o.d[0], o.d[1], o.d[2]);
      o.key = buf;
      o.index = (int)out.size();
      out.push_back(o);
    }
  }
  if (c->spread_order && out.size() > 2) {
    // processing order: farthest point first over the tool axes (from the
    // request's first orientation), each fixture set's orientations kept
    // together.  f is a minimum, so the order changes no result; spreading the
    // directions early lowers f sooner, and the bound then skips more blocks.
    const size_t n = out.size();
    std::vector<int> ord;
    std::vector<char> taken(n, 0);
    std::vector<double> far(n, 1e300);
    ord.push_back(0);
    taken[0] = 1;
    while (ord.size() < n) {
      const Orient& l = out[ord.back()];
      size_t best = n;
      for (size_t i = 0; i < n; i++) {
        if (taken[i]) continue;
        const double dot = l.d[0] * out[i].d[0] + l.d[1] * out[i].d[1] + l.d[2] * out[i].d[2];
        far[i] = std::min(far[i], 1.0 - dot);
        if (best == n || far[i] > far[best]) best = i;
      }
      taken[best] = 1;
      ord.push_back((int)best);
    }
    if (r->n_fixture_sets > 0)
      std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
        return r->fixture_of[a] < r->fixture_of[b];
      });
    std::vector<Orient> sorted;
    sorted.reserve(n);
    for (int i : ord) sorted.push_back(out[i]);
    out.swap(sorted);
  }
  return IMF_OK;
}

static void raster_desc_for(const imf_ctx* c, int tid, const Orient& o, int nd, int lattice,
                            int sharp, imf_raster_desc& d) {
  const imf_tool& t = c->tools[tid];
  std::memset(&d, 0, sizeof d);
  d.kind = t.kind;
  d.ndim = nd;
  d.lattice = lattice;
  d.sharp = sharp;
  if (t.kind == IMF_TOOL_VOXEL) {
    // image of the label box (widened by half a voxel) under R, plus one
    const imf_ctx::VoxTool& v = c->vtools[tid];
    d.vox = v.dev;
    for (int a = 0; a < 3; a++) {
      d.vdim[a] = v.dim[a];
      d.vorg[a] = v.org[a];
      d.d[a] = o.d[a];
    }
    for (int i = 0; i < 9; i++) d.R[i] = o.R[i];
    int best = 0;
    for (int a = 0; a < 3; a++) {
      double mn = 1e300, mx = -1e300;
      for (int k = 0; k < 8; k++) {
        double p = 0;
        for (int b = 0; b < 3; b++) {
          const double e = (k >> b) & 1 ? (double)(v.dim[b] - 1 - v.org[b]) + 0.5
                                        : -(double)v.org[b] - 0.5;
          p += o.R[3 * a + b] * e;
        }
        mn = std::min(mn, p);
        mx = std::max(mx, p);
      }
      d.lo[a] = (int)std::floor(mn) - 1;
      d.dim[a] = (int)std::ceil(mx) + 1 - d.lo[a] + 1;
      if (std::fabs(d.d[a]) > std::fabs(d.d[best])) best = a;
    }
    d.s_axis = best;
    return;
  }
  d.r = t.cutter_r;
  d.L = t.cutter_len;
  d.rh = t.holder_r;
  d.LH = t.cutter_len + t.holder_len;
  for (int a = 0; a < 3; a++) {
    d.d[a] = a < nd ? o.d[a] : 0.0;
    d.v[a] = a < nd ? o.v[a] : 0;
  }
  d.vn = d.v[0] * d.v[0] + d.v[1] * d.v[1] + d.v[2] * d.v[2];
  d.r2 = (long long)std::llround(2 * t.cutter_r);
  d.L2 = (long long)std::llround(2 * t.cutter_len);
  d.rh2 = (long long)std::llround(2 * t.holder_r);
  d.LH2 = (long long)std::llround(2 * (t.cutter_len + t.holder_len));
  // conservative bounding box: every tool point is a d + p, a in [0, len], |p| <= rmax
  const double len = std::max(t.cutter_len + t.holder_len, 2 * t.cutter_r);
  const double rmax = std::max(t.cutter_r, t.holder_r);
  int best = 0;
  for (int a = 0; a < 3; a++) {
    if (a >= nd) {
      d.lo[a] = 0;
      d.dim[a] = 1;
      continue;
    }
    const double e = len * d.d[a];
    const int lo = (int)std::floor(std::min(e, 0.0) - rmax) - 1;
    const int hi = (int)std::ceil(std::max(e, 0.0) + rmax) + 1;
    d.lo[a] = lo;
    d.dim[a] = hi - lo + 1;
    if (std::fabs(d.d[a]) > std::fabs(d.d[best])) best = a;
  }
  d.s_axis = best;
}

// Sharp-point runs along a lattice vector.  The minimum over S costs two
// lookups per run, and S splits into fewer runs along a short lattice vector
// near the tool axis than along a coordinate axis (a line meets a convex set
// in one run).  Among the primitive vectors with components in [-2, 2] (one of
// each +-v pair, the coordinate axes included), take the one with the fewest
// runs; keep the axis runs `ar` (along `ax`) unless another vector saves at
// least 5% of them with no run longer than 127 points (six levels).  Exact: the
// runs cover S whatever the vector.  Returns false to keep the axis runs.
// Storing one sparse-table level costs about as much as this many lookups of
// the minimum pass: one level array written over the query box vs. one gather
// per voxel of the blocks the bound keeps.  A level whose runs are few is
// cheaper left out, its runs read through more windows of a lower level.  Set
// by measurement on 256^3 x 130 (whole request: 15 / 30 / 60 / 120 ->
// 122.2 / 119.5 / 117.9 / 118.1 ms, against 125.4 with every level stored).
static const int kLevelCost = 60;

static bool lattice_runs(const imf_run* ar, int n, int ax, const int* ext, int sv[3],
                         int* maxlen, std::vector<imf_run>& out) {
  int lo[3], dim[3];
  for (int a = 0; a < 3; a++) {
    lo[a] = ext[6 + a] - 2;
    dim[a] = ext[9 + a] - ext[6 + a] + 5;
  }
  const long long vol = (long long)dim[0] * dim[1] * dim[2];
  if (n <= 0 || vol > (1LL << 26)) return false;
  std::vector<uint8_t> B((size_t)vol, 0);
  auto at = [&](int x, int y, int z) {
    return ((long long)(z - lo[2]) * dim[1] + (y - lo[1])) * dim[0] + (x - lo[0]);
  };
  std::vector<int> pts;
  for (int r = 0; r < n; r++)
    for (int j = 0; j < ar[r].len; j++) {
      int k[3] = {ar[r].x, ar[r].y, ar[r].z};
      k[ax] += j;
      B[(size_t)at(k[0], k[1], k[2])] = 1;
      pts.push_back(k[0]);
      pts.push_back(k[1]);
      pts.push_back(k[2]);
    }
  const size_t np = pts.size() / 3;
  int best = n, bv[3] = {0, 0, 0};
  for (int vz = -2; vz <= 2; vz++)
    for (int vy = -2; vy <= 2; vy++)
      for (int vx = -2; vx <= 2; vx++) {
        const int v[3] = {vx, vy, vz};
        const int f = vx ? vx : (vy ? vy : vz);
        if (f <= 0) continue;  // zero, or the negative of a listed vector
        int gd = 0;
        for (int a = 0; a < 3; a++) gd = std::gcd(gd, std::abs(v[a]));
        if (gd != 1) continue;
        if (std::abs(v[0]) + std::abs(v[1]) + std::abs(v[2]) == 1 && v[ax] != 0) continue;
        int cnt = 0;
        for (size_t i = 0; i < np && cnt < best; i++)
          cnt += !B[(size_t)at(pts[3 * i] - vx, pts[3 * i + 1] - vy, pts[3 * i + 2] - vz)];
        if (cnt < best && (double)cnt < 0.95 * n) {
          best = cnt;
          bv[0] = vx;
          bv[1] = vy;
          bv[2] = vz;
        }
      }
  if (!bv[0] && !bv[1] && !bv[2]) return false;
  auto in = [&](int x, int y, int z) {
    return x >= lo[0] && x < lo[0] + dim[0] && y >= lo[1] && y < lo[1] + dim[1] &&
           z >= lo[2] && z < lo[2] + dim[2] && B[(size_t)at(x, y, z)];
  };
  out.clear();
  int ml = 0;
  for (size_t i = 0; i < np; i++) {
    const int x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
    if (in(x - bv[0], y - bv[1], z - bv[2])) continue;
    int len = 1;
    while (in(x + len * bv[0], y + len * bv[1], z + len * bv[2])) len++;
    if (len > 127) return false;
    ml = std::max(ml, len);
    out.push_back(imf_run{x, y, z, len});
  }
  for (int a = 0; a < 3; a++) sv[a] = bv[a];
  *maxlen = ml;
  return true;
}

static int rows_of(const imf_raster_desc& d) {
  const int u = (d.s_axis + 1) % 3, w = (d.s_axis + 2) % 3;
  return std::max(d.dim[1] * d.dim[2], d.dim[u] * d.dim[w]);
}

// Rasterize every orientation of `os` that is not cached yet.
static imf_status ensure_rasters(imf_ctx* c, const imf_request* r, const std::vector<Orient>& os,
                                 hipStream_t s) {
  std::vector<const Orient*> miss;
  std::map<std::string, int> seen;
  for (auto& o : os)
    if (!c->rasters.count(o.key) && !seen.count(o.key)) {
      seen[o.key] = 1;
      miss.push_back(&o);
    }
  if (miss.empty()) return IMF_OK;
  const int n = (int)miss.size();
  std::vector<imf_raster_desc> hd(n);
  long long flags_total = 0, rows_total = 0;
  int max_vol = 0, max_rows = 0;
  for (int i = 0; i < n; i++) {
    raster_desc_for(c, miss[i]->tool, *miss[i], r->ndim, r->dir_kind == IMF_DIR_LATTICE,
                    r->sharp, hd[i]);
    const long long vol = (long long)hd[i].dim[0] * hd[i].dim[1] * hd[i].dim[2];
    if (vol > (1LL << 30)) return fail(IMF_EINVAL, "tool raster box too large");
    hd[i].flags_off = flags_total;
    flags_total += (vol + 3) & ~3LL;
    hd[i].rows_off = rows_total;
    const int rw = rows_of(hd[i]);
    rows_total += rw;
    max_vol = std::max(max_vol, (int)vol);
    max_rows = std::max(max_rows, rw);
  }
  imf_raster_desc* dd = nullptr;
  uint8_t* flags = nullptr;
  int* ext = nullptr;
  imf_run* slots = nullptr;
  int* cnt = nullptr;
  long long* base = nullptr;
  imf_run* pool = nullptr;
  auto cleanup = [&]() {
    hipFree(dd);
    hipFree(flags);
    hipFree(ext);
    hipFree(slots);
    hipFree(cnt);
    hipFree(base);
  };
  std::vector<int> hext((size_t)n * IMF_EXT_INTS);
  for (int i = 0; i < n; i++) {
    int* e = &hext[(size_t)i * IMF_EXT_INTS];
    for (int a = 0; a < IMF_EXT_INTS; a++) e[a] = 0;
    for (int a = 0; a < 3; a++) {
      e[a] = e[6 + a] = 1 << 29;
      e[3 + a] = e[9 + a] = -(1 << 29);
    }
  }
  hipError_t he = hipSuccess;
  if ((he = hipMalloc(&dd, sizeof(imf_raster_desc) * n)) == hipSuccess &&
      (he = hipMalloc(&flags, flags_total)) == hipSuccess &&
      (he = hipMalloc(&ext, sizeof(int) * hext.size())) == hipSuccess &&
      (he = hipMalloc(&slots, sizeof(imf_run) * rows_total * 3 * IMF_MAX_RUNS_PER_ROW)) ==
          hipSuccess &&
      (he = hipMalloc(&cnt, sizeof(int) * rows_total * 3)) == hipSuccess &&
      (he = hipMalloc(&base, sizeof(long long) * n * 3)) == hipSuccess) {
  }
  if (he != hipSuccess) {
    cleanup();
    return fail(IMF_ENOMEM, "raster workspace: %s", hipGetErrorString(he));
  }
#define RCHK(call)                                                                        \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) {                                                               \
      cleanup();                                                                          \
      return fail(IMF_EDEVICE, "%s: %s", #call, hipGetErrorString(e_));                   \
    }                                                                                     \
  } while (0)
  RCHK(hipMemcpyAsync(dd, hd.data(), sizeof(imf_raster_desc) * n, hipMemcpyHostToDevice, s));
  RCHK(hipMemcpyAsync(ext, hext.data(), sizeof(int) * hext.size(), hipMemcpyHostToDevice, s));
  RCHK(imf_launch_raster(dd, n, max_vol, flags, ext, s));
  RCHK(imf_launch_sharp_subset(dd, n, max_vol, flags, ext, s));
  RCHK(imf_launch_runs(dd, n, max_rows, flags, slots, cnt, ext, s));
  RCHK(hipMemcpyAsync(hext.data(), ext, sizeof(int) * hext.size(), hipMemcpyDeviceToHost, s));
  RCHK(hipStreamSynchronize(s));
  std::vector<long long> hb((size_t)n * 3);
  long long total = 0;
  for (int i = 0; i < n; i++) {
    const int* e = &hext[(size_t)i * IMF_EXT_INTS];
    if (e[14]) {
      cleanup();
      return fail(IMF_EINVAL, "tool raster has more than %d runs in a row", IMF_MAX_RUNS_PER_ROW);
    }
    if (e[12] <= 0 || e[13] <= 0) {
      cleanup();
      return fail(IMF_EINVAL, "oriented tool %s has no voxels or no sharp points",
                  miss[i]->key.c_str());
    }
    for (int k = 0; k < 3; k++) {
      hb[(size_t)i * 3 + k] = total;
      total += e[15 + k];
    }
  }
  if (hipMalloc(&pool, sizeof(imf_run) * std::max(total, 1LL)) != hipSuccess) {
    cleanup();
    return fail(IMF_ENOMEM, "raster run pool");
  }
  c->raster_pools.push_back(pool);
  c->raster_bytes += sizeof(imf_run) * std::max(total, 1LL);
  RCHK(hipMemcpyAsync(base, hb.data(), sizeof(long long) * hb.size(), hipMemcpyHostToDevice, s));
  RCHK(imf_launch_compact(dd, n, max_rows, slots, cnt, base, pool, s));
  RCHK(hipStreamSynchronize(s));
  // sharp-point runs along lattice vectors (3D): chosen on the host from the
  // axis runs, uploaded as one more pool
  std::vector<OrientEntry> ents(n);
  for (int i = 0; i < n; i++) {
    OrientEntry& e = ents[i];
    std::memcpy(e.ext, &hext[(size_t)i * IMF_EXT_INTS], sizeof e.ext);
    e.s_axis = hd[i].s_axis;
    for (int a = 0; a < 3; a++) e.sv[a] = a == e.s_axis;
    e.maxlen = e.ext[9 + e.s_axis] - e.ext[6 + e.s_axis] + 1;
    e.truns = pool + hb[(size_t)i * 3 + 0];
    e.sruns = pool + hb[(size_t)i * 3 + 1];
    e.sxruns = pool + hb[(size_t)i * 3 + 2];
  }
  {
    std::vector<imf_run> hpool((size_t)std::max(total, 1LL));
    RCHK(hipMemcpy(hpool.data(), pool, sizeof(imf_run) * hpool.size(), hipMemcpyDeviceToHost));
    std::vector<imf_run> vall, one;
    std::vector<long long> voff(n, -1);
    for (int i = 0; i < n; i++) {
      OrientEntry& e = ents[i];
      const imf_run* ar = hpool.data() + hb[(size_t)i * 3 + 1];
      int sv[3], ml = 0;
      if (r->ndim == 3 && c->lattice_runs &&
          lattice_runs(ar, e.ext[16], e.s_axis, e.ext, sv, &ml, one)) {
        e.s_axis = std::abs(sv[0]) + std::abs(sv[1]) + std::abs(sv[2]) == 1
                       ? (sv[0] ? 0 : (sv[1] ? 1 : 2))
                       : 3;
        for (int a = 0; a < 3; a++) e.sv[a] = e.s_axis < 3 ? (a == e.s_axis) : sv[a];
        e.ext[16] = (int)one.size();
        e.maxlen = ml;
      } else {
        one.assign(ar, ar + e.ext[16]);
      }
      // A run of length l is read through windows of one sparse-table level
      // s <= floor(log2 l): ceil(l / 2^s) windows of length 2^s, the last
      // one ending at the run's end (two when s = floor(log2 l), one when
      // l = 2^s).  Each window is itself a run of S (min is idempotent, so
      // overlaps are harmless): splitting every run into its windows leaves
      // runs of power-of-two length only, one lookup each, which are then
      // ordered by level and by first point (z, y, x), so that consecutive
      // lookups of the gather loop read the same level array at neighbouring
      // lines.  Which levels to store is chosen per orientation (see
      // kLevelCost).  Kept whole if the windows would not fit the minimum
      // pass's LDS staging.
      auto pow2 = [](const imf_run& u) { return (u.len & (u.len - 1)) == 0; };
      auto level = [](const imf_run& u) { return 31 - __builtin_clz((unsigned)u.len); };
      {
        int hist[128] = {0}, top = 0;
        bool fits = true;
        for (const imf_run& u : one) {
          if (u.len > 127) fits = false;
          else hist[u.len]++;
          top = std::max(top, level(u));
        }
        // windows of a run of length l with the stored levels `lv` (bit s-1:
        // level s) and the total cost of a choice
        auto read_level = [](int l, unsigned lv) {
          int s = 31 - __builtin_clz((unsigned)l);
          while (s > 0 && !((lv >> (s - 1)) & 1u)) s--;
          return s;
        };
        auto windows = [&](unsigned lv, unsigned* used) {
          long long n = 0;
          unsigned u = 0;
          for (int l = 1; l < 128; l++)
            if (hist[l]) {
              const int s = read_level(l, lv), w = 1 << s;
              n += (long long)hist[l] * ((l + w - 1) / w);
              if (s > 0) u |= 1u << (s - 1);
            }
          if (used) *used = u;
          return n;
        };
        const unsigned all = top > 0 ? (1u << top) - 1 : 0u;
        unsigned pick = all;
        if (fits) {
          long long best = -1;
          for (unsigned lv = 0; lv <= all; lv++) {
            unsigned used;
            const long long n = windows(lv, &used);
            const long long cost = n + (long long)kLevelCost * __builtin_popcount(used);
            if (n <= IMF_MF_LDS_RUNS && (best < 0 || cost < best)) {
              best = cost;
              pick = lv;
            }
          }
          if (best < 0) fits = false;  // even the fewest windows overflow
        }
        if (fits) {
          std::vector<imf_run> win;
          win.reserve((size_t)windows(pick, nullptr));
          int ml = 1;
          for (const imf_run& u : one) {
            const int w = 1 << read_level(u.len, pick);
            ml = std::max(ml, w);
            for (int o = 0; o < u.len; o += w) {
              const int sh = std::min(o, u.len - w);
              win.push_back(imf_run{u.x + sh * e.sv[0], u.y + sh * e.sv[1], u.z + sh * e.sv[2], w});
            }
          }
          one.swap(win);
          e.ext[16] = (int)one.size();
          e.maxlen = ml;
        }
      }
      std::sort(one.begin(), one.end(), [&](const imf_run& p, const imf_run& q) {
        if (pow2(p) != pow2(q)) return pow2(p);
        if (level(p) != level(q)) return level(p) < level(q);
        return p.z != q.z ? p.z < q.z : (p.y != q.y ? p.y < q.y : p.x < q.x);
      });
      e.n_pow2 = (int)std::count_if(one.begin(), one.end(), pow2);
      // a run of length l reads level floor(log2 l) only; the level passes
      // skip the stores of levels no run reads
      e.lvl_used = 0;
      for (const imf_run& u : one)
        if (u.len >= 2) e.lvl_used |= 1u << (30 - __builtin_clz((unsigned)u.len));
      voff[i] = (long long)vall.size();
      vall.insert(vall.end(), one.begin(), one.end());
    }
    if (!vall.empty()) {
      imf_run* vpool = nullptr;
      if (hipMalloc(&vpool, sizeof(imf_run) * vall.size()) != hipSuccess) {
        cleanup();
        return fail(IMF_ENOMEM, "raster run pool");
      }
      c->raster_pools.push_back(vpool);
      c->raster_bytes += sizeof(imf_run) * vall.size();
      RCHK(hipMemcpy(vpool, vall.data(), sizeof(imf_run) * vall.size(), hipMemcpyHostToDevice));
      for (int i = 0; i < n; i++)
        if (voff[i] >= 0) ents[i].sruns = vpool + voff[i];
    }
  }
#undef RCHK
  for (int i = 0; i < n; i++) c->rasters[miss[i]->key] = ents[i];
  cleanup();
  return IMF_OK;
}

// ---------------------------------------------------------------------------
// planning
// ---------------------------------------------------------------------------
static const int kFpCap = 16384;  // footprint cells per orientation
// Bracket entries per orientation above which the inverse x pass defers its
// appends (measured: 256^3 x 130 lists about 2e3 per orientation, faster
// appended at once; 384^3 x 512 in a TO loop about 2e5, whose x pass takes
// 147 instead of 219 ms per iteration with the appends deferred).
static const double kDeferListed = 2e4;

struct Plan {
  int nd, n[3];
  long long N;
  int words;
  int method;  // FFT or DIRECT
  int P[3];
  imf_fft_len fl[3];
  int B;
  int nO;
  std::vector<imf_orient_desc> desc;
  std::vector<imf_orient_desc> sweep_desc;
  std::vector<const OrientEntry*> ent;
  std::vector<std::string> keys;
  int max_m[3];
  long long max_vol;
  int max_t[3];
  int nlvl;
  bool theta_known, two_phase, masks, sweep, cache, bnb;
  int shape;
  long long cell_stride, nblocks, cell_waves, nwords_blk;
  int tuned_batch = 8, tuned_shape = 2, wg_per_cu = 8;  // launch parameters in effect
  int fft_plan = 0;  // inverse transform plans: z | y << 2 | x << 4 (imf_inv_args.fplan)
  // batches: orientations [bstart[b], bstart[b+1]), all seeing fixture set bset[b]
  // (0 without fixture sets); at most B wide, split wherever the set changes
  std::vector<int> bstart, bset;
  int nsets = 0;  // fixture sets (0: the common fixture only)
  int debug_pos = -1;  // processing position of the orientation whose overlaps are copied
  double theta;
  double band;
  // Exact decisions at the threshold theta_B = lambda F_max of B (and of
  // two-phase masks).  E bounds |g32 - g| (voxel units; 0 for binary); scale
  // is the fixed-point unit (2^-24 for density, 1 for binary).  thB_known:
  // theta_B is known before the request runs (lambda = 0, or a second pass
  // given the exact F_max) and the first-pass recheck decides it too;
  // otherwise (exact) F_max is found exactly after all orientations and the
  // band around theta_B is decided from the stored overlaps (gst) or, without
  // room for them, by a second pass.
  double E = 0, scale = 1;
  bool thB_known = true;
  double thB = 0;                 // theta_B in voxel units when known
  unsigned long long known_Fq = 0;
  bool known = false;             // a second pass: F_max given
  bool exact = false;             // F_max and the band decided after the first pass
  bool gam = false;               // gamma stack (two-phase masks or exact)
  bool intmask = false;           // masks at theta_B in the workspace (exact, no such output)
  bool gst = false;               // g of every orientation kept (band scan)
  // gamma stack of the kept blocks only (with the bound): gcap floats, sized
  // from the kept fraction of the last request of this shape (gkey)
  bool gcomp = false;
  long long gcap = 0;
  std::string gkey;
  int band_cap = 0, cand_cap = 0;
  // an expected threshold (the last exact F_max of this request shape): the
  // inverse x pass lists the overlaps of the bracket (blo, bhi] (voxel units),
  // which replaces the band scan (or the second pass) when it holds the band
  std::string hint_key;
  bool hinted = false;
  double blo = 0, bhi = 0, hint_delta = 0;
  double hint_pred = 0;  // the expected F_max (fixed point)
  // the inverse x pass writes its bracket (and guard-band) entries after its
  // rows, one reservation per wave: the last bracket of this shape was long
  bool defer_appends = false;
  // workspace layout (bytes)
  size_t ws_bytes;
  long long spec_elems;
};

static imf_status validate(const imf_request* r) {
  if (!r) return fail(IMF_EINVAL, "request is NULL");
  if (r->ndim != 2 && r->ndim != 3) return fail(IMF_EINVAL, "ndim must be 2 or 3");
  if (r->nx < 1 || r->ny < 1 || r->nz < 1) return fail(IMF_EINVAL, "empty grid");
  if (r->ndim == 2 && r->nz != 1) return fail(IMF_EINVAL, "2D grids need nz = 1");
  if (r->nx > 1024 || r->ny > 1024 || r->nz > 1024)
    return fail(IMF_EINVAL, "grid larger than 1024 per axis");
  if (!r->design) return fail(IMF_EINVAL, "design is NULL");
  if (r->n_tools < 1 || !r->tool_ids || !r->n_dirs || !r->dirs)
    return fail(IMF_EINVAL, "no tools or directions");
  if (r->sharp < 0 || r->sharp > 2) return fail(IMF_EINVAL, "unknown sharp-point mode");
  if (!(r->lambda >= 0 && r->lambda < 1)) return fail(IMF_EINVAL, "lambda must be in [0, 1)");
  if (!std::isfinite(r->tau)) return fail(IMF_EINVAL, "tau is not finite");
  if (r->method < 0 || r->method > 2) return fail(IMF_EINVAL, "unknown method");
  if (r->batch < 0 || r->batch > 64) return fail(IMF_EINVAL, "batch must be in [0, 64]");
  if (r->n_fixture_sets < 0 || r->n_fixture_sets > 256)
    return fail(IMF_EINVAL, "n_fixture_sets must be in [0, 256]");
  if (r->n_fixture_sets > 0) {
    if (!r->fixture_sets || !r->fixture_of)
      return fail(IMF_EINVAL, "fixture sets need fixture_sets and fixture_of");
    long long nO = 0;
    for (int i = 0; i < r->n_tools; i++) nO += std::max(r->n_dirs[i], 0);
    for (long long q = 0; q < nO; q++)
      if (r->fixture_of[q] < 0 || r->fixture_of[q] >= r->n_fixture_sets)
        return fail(IMF_EINVAL, "fixture_of[%lld] = %d is not a fixture set", q,
                    r->fixture_of[q]);
  }
  return IMF_OK;
}

static std::string tune_key(const Plan& p) {
  char key[96];
  snprintf(key, sizeof key, "%d|%d,%d,%d|%d,%d,%d", p.method, p.n[0], p.n[1], p.n[2], p.P[0],
           p.P[1], p.P[2]);
  return key;
}

// launch parameters for a plan: the autotuned ones for its shape if any, else
// the context defaults; a candidate being timed by the autotuner overrides both
static void ctx_tuned_params(imf_ctx* c, Plan& p) {
  p.tuned_batch = 8;
  p.fft_plan = p.method == IMF_METHOD_FFT ? imf_fft_default_plan(p.P[2], p.P[1], p.P[0]) : 0;
  p.tuned_shape = c->mf_shape;
  p.wg_per_cu = c->mf_wg_per_cu;
  auto it = c->tuned.find(tune_key(p));
  if (it != c->tuned.end()) {
    p.tuned_batch = it->second.batch;
    if (it->second.shape >= 0) p.tuned_shape = it->second.shape;
    if (it->second.wg > 0) p.wg_per_cu = it->second.wg;
    p.fft_plan = it->second.fft;
  }
  if (c->force_shape >= 0) p.tuned_shape = c->force_shape;
  if (c->force_wg > 0) p.wg_per_cu = c->force_wg;
  if (c->force_fft >= 0) p.fft_plan = c->force_fft;
}

static imf_status make_plan(imf_ctx* c, const imf_request* r, const imf_outputs* out,
                            const std::vector<Orient>& os, Plan& p,
                            const unsigned long long* known_Fq = nullptr) {
  p.nd = r->ndim;
  p.n[0] = r->nx;
  p.n[1] = r->ny;
  p.n[2] = r->nz;
  p.N = (long long)r->nx * r->ny * r->nz;
  p.words = (r->nx + 63) / 64;
  p.nO = (int)os.size();
  p.desc.resize(p.nO);
  p.ent.resize(p.nO);
  p.keys.resize(p.nO);
  long long need[3] = {1, 1, 1};
  for (int a = 0; a < 3; a++) {
    p.max_m[a] = 1;
    p.max_t[a] = 1;
  }
  p.max_vol = 1;
  int max_sdim = 1;
  for (int q = 0; q < p.nO; q++) {
    const OrientEntry& e = c->rasters.at(os[q].key);
    p.ent[q] = &e;
    p.keys[q] = os[q].key;
    imf_orient_desc& d = p.desc[q];
    std::memset(&d, 0, sizeof d);
    long long vol = 1;
    for (int a = 0; a < 3; a++) {
      const int omin = e.ext[a], omax = e.ext[3 + a], kmin = e.ext[6 + a], kmax = e.ext[9 + a];
      d.box_lo[a] = -kmax;
      d.box_dim[a] = p.n[a] + kmax - kmin;
      d.tlo[a] = omin;
      d.tdim[a] = omax - omin + 1;
      need[a] = std::max(need[a], (long long)p.n[a] + std::max(kmax - omin, omax - kmin));
      p.max_m[a] = std::max(p.max_m[a], d.box_dim[a]);
      p.max_t[a] = std::max(p.max_t[a], d.tdim[a]);
      vol *= d.box_dim[a];
    }
    p.max_vol = std::max(p.max_vol, vol);
    d.s_axis = e.s_axis;
    for (int a = 0; a < 3; a++) d.sv[a] = e.sv[a];
    d.n_sruns = e.ext[16];
    d.n_sruns1 = e.n_pow2;
    d.lvl_used = e.lvl_used;
    d.n_truns = e.ext[15];
    d.sruns = e.sruns;
    d.truns = e.truns;
    d.spec = nullptr;
    d.out_q = os[q].index;
    if (out && out->debug_overlap && os[q].index == out->debug_orient) p.debug_pos = q;
    const int sdim = e.maxlen;  // longest run of S
    max_sdim = std::max(max_sdim, sdim);
    d.nlvl = 0;
    while ((2 << d.nlvl) <= sdim) d.nlvl++;
  }
  if (p.max_vol > (1LL << 31) - 1) return fail(IMF_EINVAL, "query box too large");
  p.nlvl = 0;
  while ((2 << p.nlvl) <= max_sdim) p.nlvl++;
  // method
  p.method = r->method;
  if (p.method == IMF_METHOD_AUTO) p.method = (p.nd == 2 || p.N <= 32 * 32 * 32) ? IMF_METHOD_DIRECT : IMF_METHOD_FFT;
  for (int a = 0; a < 3; a++) {
    p.P[a] = 1;
    p.fl[a] = make_len(1);
  }
  if (p.method == IMF_METHOD_FFT) {
    for (int a = 0; a < p.nd; a++) {
      const int m = imf_fft_size((int)need[a]);
      if (m < 0) return fail(IMF_EINVAL, "transform length %lld along axis %d exceeds 1024",
                             need[a], a);
      p.P[a] = m;
      p.fl[a] = make_len(m);
    }
  }
  // batch width
  const bool plain = (r->flags & IMF_FLAG_PLAIN) != 0;
  p.B = r->batch;
  ctx_tuned_params(c, p);
  if (p.B == 0) p.B = p.tuned_batch;
  if (plain) p.B = 1;
  p.B = std::max(1, std::min(p.B, p.nO));
  p.nsets = r->n_fixture_sets;
  p.bstart.assign(1, 0);
  p.bset.clear();
  for (int q = 0; q < p.nO;) {
    const int set = p.nsets ? r->fixture_of[os[q].index] : 0;
    int e = q + 1;
    while (e < p.nO && e - q < p.B && (!p.nsets || r->fixture_of[os[e].index] == set)) e++;
    for (int k = q; k < e; k++) p.desc[k].set = set;
    p.bset.push_back(set);
    p.bstart.push_back(e);
    q = e;
  }
  // thresholds
  p.masks = out && out->acc_masks;
  p.sweep = p.masks && (r->flags & IMF_FLAG_MASK_SWEEP);
  p.cache = p.method == IMF_METHOD_FFT && !plain && !(r->flags & IMF_FLAG_NO_CACHE);
  if (r->mask_theta_abs >= 0) {
    p.theta_known = true;
    p.theta = r->mask_theta_abs;
  } else if (r->lambda == 0) {
    p.theta_known = true;
    p.theta = 0;
  } else {
    p.theta_known = false;
    p.theta = 0;
  }
  p.two_phase = p.masks && !p.theta_known;
  if (p.two_phase && p.sweep)
    return fail(IMF_EINVAL, "the sweep mask route needs a known threshold (mask_theta_abs >= 0 or lambda = 0)");
  // Error model of the float32 overlaps (density; binary overlaps are rounded
  // to exact integers).  Transform path: the error of a float32 transform
  // correlation is relative to the magnitude of its outputs, at most |T|
  // (rho <= 1), growing like the square root of the number of radix stages;
  // E = 8 u sqrt(log2 P^3) |T| (u = 2^-24) holds measured errors with a
  // margin of about ten (256^3 x 130: largest of 10^5 sampled errors 8.5e-3,
  // E = 0.097), and every exact recomputation checks it (IMF_EACCURACY when
  // one exceeds E / 2).  Direct path: exact sums rounded once to float32,
  // |g32 - g| <= 2^-24 |T|.
  p.E = 0;
  p.scale = r->design_is_density ? 1.0 / 16777216.0 : 1.0;
  if (r->design_is_density) {
    long long maxT = 1;
    for (auto* e : p.ent) maxT = std::max<long long>(maxT, e->ext[12]);
    const double u = 1.0 / 16777216.0;
    if (p.method == IMF_METHOD_FFT) {
      const double lg = std::log2((double)p.P[0] * p.P[1] * p.P[2]);
      p.E = 8.0 * u * std::sqrt(lg) * (double)maxT;
    } else {
      p.E = u * (double)maxT;
    }
  }
  p.band = p.E;  // half-width of the first-pass recheck around a known threshold
  // the threshold of B
  p.known = known_Fq != nullptr;
  p.known_Fq = known_Fq ? *known_Fq : 0;
  p.thB_known = r->lambda == 0 || p.known || !r->design_is_density;
  p.thB = p.known ? r->lambda * (double)p.known_Fq * p.scale : 0.0;
  p.exact = r->design_is_density && !p.thB_known;
  p.gam = p.two_phase || p.exact;
  p.intmask = p.exact && !p.two_phase;
  // expected threshold: transform path, no first-pass recheck (the listed
  // values are the ones the minimum pass reads)
  p.hinted = false;
  if (p.exact && p.method == IMF_METHOD_FFT && !p.theta_known) {
    std::string k;
    auto put = [&](const void* v, size_t n) { k.append((const char*)v, n); };
    const long long ki[] = {r->nx, r->ny, r->nz, r->dir_kind, r->sharp, r->n_tools,
                            r->n_fixture_sets};
    put(ki, sizeof ki);
    put(&r->lambda, sizeof(double));
    const void* kp[] = {r->fixture, r->domain, r->fixture_sets};
    put(kp, sizeof kp);
    for (const auto& key : p.keys) k += key + "|";
    if (r->n_fixture_sets) put(r->fixture_of, sizeof(int) * (size_t)p.nO);
    p.hint_key = k;
    auto it = c->hints.find(k);
    if (c->use_hints && it != c->hints.end()) {
      // the next maximum extrapolated from the last two (a TO loop's design
      // drifts), the bracket as wide as recent predictions erred (twice)
      const imf_ctx::Hint& h = it->second;
      double pred = (double)h.F[0];
      if (h.F[2]) {  // a drift over the last three continues by its mean step
        const double d1 = (double)h.F[0] - (double)h.F[1], d2 = (double)h.F[1] - (double)h.F[2];
        if (d1 * d2 > 0) pred = std::max(0.0, (double)h.F[0] + 0.5 * (d1 + d2));
      }
      p.hinted = true;
      p.hint_pred = pred;
      p.hint_delta = h.delta;
      p.defer_appends = c->defer_mode < 0 && h.listed > kDeferListed;
      const double th = r->lambda * pred * p.scale;
      p.blo = th * (1.0 - p.hint_delta) - p.E;
      p.bhi = th * (1.0 + p.hint_delta) + p.E;
    }
  }
  if (c->defer_mode == 1) p.defer_appends = true;
  if (p.known && p.two_phase) {  // second pass: the masks' threshold is theta_B
    p.two_phase = false;
    p.gam = false;
    p.theta_known = true;
    p.theta = p.thB;
  }
  // branch and bound for the sharp-point minimum (not in the plain comparator)
  p.bnb = !plain && !(r->flags & IMF_FLAG_NO_BOUND) && p.N >= c->bound_min_voxels;
  p.shape = p.nd == 2 ? 0 : p.tuned_shape;
  {
    int wx, wy, wz;
    imf_block_dims(p.shape, wx, wy, wz);
    const long long nbx = (r->nx + wx - 1) / wx, nby = (r->ny + wy - 1) / wy,
                    nbz = (r->nz + wz - 1) / wz;
    p.nblocks = nbx * nby * nbz;
    p.nwords_blk = (imf_block_logical(p.shape, r->nx, r->ny, r->nz) + 63) / 64;
    // work lists hold packed block coordinates
    if (nbx >= 1024 || nby >= 2048 || nbz >= 2048) p.bnb = false;
    // the gamma stack holds the blocks the bound keeps, 64 values each, at a
    // capacity of 1.25 times the kept fraction seen last time for this shape
    // (half the blocks before that); above 80% the full stack is kept.  Where
    // the full stack is small against the budget it is kept too: the compact
    // one costs a slot lookup per value in the mask pass (256^3 x 130, 8.7 GB
    // of full stack: +0.8 ms per request)
    const bool big = 4.0 * (double)p.nO * (double)r->nx * r->ny * r->nz > (double)c->budget / 16;
    if (p.gam && p.bnb && c->compact_gamma > 0 && (big || c->compact_forced)) {
      char k[64];
      snprintf(k, sizeof k, "|%d|%d", p.nO, p.shape);
      p.gkey = tune_key(p) + k;
      auto it = c->gkept.find(p.gkey);
      const double fr = it == c->gkept.end() ? c->compact_gamma
                                             : std::min(1.0, 1.25 * it->second + 0.01);
      const long long full = (long long)p.nO * p.nblocks;
      p.gcomp = fr < 0.8 && full < (1LL << 40);
      p.gcap = p.gcomp ? 64 * (long long)std::ceil(fr * (double)full) : 0;
    }
    p.cell_stride = 1;
    p.cell_waves = 1;
    for (int q = 0; q < p.nO; q++) {
      const imf_orient_desc& d = p.desc[q];
      const long long cdx = (d.box_dim[0] + wx - 1) / wx + 1;
      const long long cdy = (d.box_dim[1] + wy - 1) / wy + 1;
      const long long cdz = (d.box_dim[2] + wz - 1) / wz + 1;
      p.cell_stride = std::max(p.cell_stride, cdx * cdy * cdz);
      p.cell_waves = std::max(p.cell_waves, (cdx * wx + 63) / 64 * cdy * ((cdz + 7) / 8));
    }
  }
  const int h = p.P[0] / 2 + 1;
  p.spec_elems = (long long)p.P[1] * h * p.P[2];
  // workspace
  size_t b = 0;
  auto add = [&](size_t bytes) { b += align256(bytes); };
  const long long N = p.N;
  add(sizeof(float) * N);                              // f
  add(N);                                              // omega0
  const int nps = std::max(p.nsets, 1);
  add(sizeof(long long) * (r->nx + 1) * (long long)r->ny * r->nz * nps);  // prefix sums
  if (p.nsets) add((size_t)N * (p.nsets + 1));       // fixture of each setup, union
  add(256);                                            // fmax + max_err
  const int nb = (int)p.bset.size();
  add(sizeof(int) * (nb + 1));                         // per-batch flag counters
  add(sizeof(int2) * (size_t)(1 << 20));               // flag list
  add(sizeof(imf_orient_desc) * p.nO * 2);             // descriptors (+ sweep)
  add(sizeof(float) * p.B * p.max_vol);                // g
  add(sizeof(float) * p.B * std::max(p.nlvl, 1) * p.max_vol);  // levels
  if (p.gam) add(sizeof(float) * (p.gcomp ? p.gcap : N * p.nO));  // gamma stack
  if (p.gcomp) {
    add(sizeof(long long) * p.nO);                     // each orientation's first slot
    add(sizeof(int) * (size_t)p.nO * p.nwords_blk);    // list offsets per 64 blocks
  }
  if (p.intmask) add(sizeof(uint64_t) * p.nO * (long long)r->nz * r->ny * p.words);  // masks at theta_B
  if (p.exact) {
    p.cand_cap = 1 << 16;
    // room for 16384 bracket entries per list (64 lists per orientation)
    p.band_cap = (int)std::min<long long>(std::max<long long>(1LL << 20, (long long)p.nO *
                                                                          IMF_BR_SLICES * 16384),
                                          1LL << 29);
    add(sizeof(int) * (size_t)p.cand_cap);               // candidates of the maximum
    add(sizeof(unsigned long long) * (size_t)p.cand_cap);  // their exact f
    add(sizeof(int4) * (size_t)p.band_cap);              // band entries
    add(sizeof(unsigned) * (size_t)p.nO * IMF_BR_SLICES);  // bracket list counts
    add(sizeof(uint64_t) * (size_t)r->nz * r->ny * p.words);  // Omega_0 as row bits
  }
  if (p.bnb) {
    add(sizeof(float) * p.B * p.cell_stride);           // cell minima
    add(sizeof(int) * p.B * (long long)(kFpCap + 1));   // footprints
    add(sizeof(float) * p.nblocks);                     // block maxima of f
    add(sizeof(int) * p.B * p.nblocks);                 // work lists
    add(sizeof(int) * p.B);                             // list lengths
    add(sizeof(int) * p.nO);                            // kept blocks per orientation
    add(sizeof(uint64_t) * p.B * p.nwords_blk);         // kept-block bits
    add(sizeof(int) * p.B * p.nwords_blk);              // list offsets
    if (p.gam) add(sizeof(uint64_t) * p.nO * p.nwords_blk);  // kept-block bits per orientation
  }
  if (p.sweep) add(sizeof(uint64_t) * p.B * ((p.max_m[0] + 63) / 64) * (long long)p.max_m[1] * p.max_m[2]);
  if (p.method == IMF_METHOD_FFT) {
    add(sizeof(float2) * p.spec_elems * nps);                            // rho_hat per set
    add(sizeof(float2) * (long long)r->nz * r->ny * h);                  // fwd work1
    add(sizeof(float2) * (long long)r->nz * p.P[1] * h);                 // fwd work2
    add(sizeof(float2) * p.B * (long long)p.max_t[2] * p.max_t[1] * h);  // tool work1
    add(sizeof(float2) * p.B * (long long)p.max_t[2] * p.P[1] * h);      // tool work2
    add(sizeof(float2) * p.B * p.spec_elems);                            // batch spectra
    add(sizeof(float2) * p.B * (long long)p.max_m[2] * p.P[1] * h);      // inverse w1
    add(sizeof(float2) * p.B * (long long)p.max_m[2] * p.max_m[1] * h);  // inverse w2
    add(sizeof(imf_orient_desc) * (size_t)nb * p.B);                      // per-batch miss lists
  }
  // the overlaps of every orientation (instead of one batch's) when there is
  // room beside the cached spectra of the request: the band around theta_B is
  // then read from them once F_max is known
  p.gst = false;
  if (p.exact && c->overlap_stack) {
    const size_t extra = sizeof(float) * (size_t)(p.nO - p.B) * (size_t)p.max_vol;
    const size_t spectra = p.cache ? (size_t)p.nO * 8 * (size_t)p.spec_elems : 0;
    if (b + extra + spectra + c->raster_bytes + (size_t)(1 << 30) <= c->budget) {
      p.gst = true;
      b += align256(extra);
    }
  }
  p.ws_bytes = b + 4096;
  return IMF_OK;
}

extern "C" imf_status imf_query_footprint(imf_ctx* c, const imf_request* r, size_t* bytes) {
  if (!c || !bytes) return fail(IMF_EINVAL, "NULL argument");
  STCHK(validate(r));
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  HIPCHK(hipSetDevice(c->device));
  std::vector<Orient> os;
  STCHK(enumerate(c, r, os));
  STCHK(ensure_rasters(c, r, os, c->internal));
  Plan p;
  imf_outputs o{};
  STCHK(make_plan(c, r, &o, os, p));
  *bytes = p.ws_bytes;
  return IMF_OK;
}

// cost model of the algorithmic HBM traffic (bytes) of one request
static double model_bytes(const Plan& p) {
  const double S = 8.0 * p.spec_elems;
  double tot = 0;
  for (int q = 0; q < p.nO; q++) {
    const imf_orient_desc& d = p.desc[q];
    const double M3 = (double)d.box_dim[0] * d.box_dim[1] * d.box_dim[2];
    if (p.method == IMF_METHOD_FFT) {
      const double fz = (double)d.box_dim[2] / p.P[2], fy = (double)d.box_dim[1] / p.P[1];
      tot += S + S / p.B + 2 * S * fz + 2 * S * fz * fy;
    }
    tot += 4 * M3 + 4 * M3;         // write g, read g in the min filter
    tot += 8.0 * p.N / p.B;          // running min read + write
    if (p.masks) tot += p.N / 8.0;   // mask bits
  }
  tot += 13.0 * p.N;                 // finalize
  return tot;
}

// ---------------------------------------------------------------------------
// compute
// ---------------------------------------------------------------------------
// Events on the request's stream between kernel classes.  Without profiling
// only the class boundaries of the coarse phases are marked.
struct Timer {
  std::vector<hipEvent_t> ev;
  std::vector<int> cls;
  hipStream_t s;
  bool fine = false;
  bool off = false;  // no event marks (graph capture and replay)
  void mark(int k) {
    if (off) return;
    static const bool coarse_mark[16] = {1, 1, 1, 0, 0, 1, 0, 0, 1, 1, 0, 1, 1, 1, 1, 0};
    if (!fine && !coarse_mark[k & 15]) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    if (hipEventRecord(e, s) != hipSuccess) {
      hipEventDestroy(e);
      return;
    }
    ev.push_back(e);
    cls.push_back(k);
  }
  void collect(imf_stats* st) {
    static const int coarse[16] = {0, 6, 1, 2, 2, 2, 3, 3, 3, 4, 5, 5, 5, 6, 6, 5};
    for (size_t i = 1; i < ev.size(); i++) {
      float ms = 0;
      hipEventElapsedTime(&ms, ev[i - 1], ev[i]);
      const int k = cls[i];
      if (k < 0 || k > 15) continue;
      st->t_ms[coarse[k]] += ms;
      if (fine) {
        st->k_ms[k] += ms;
        st->k_n[k] += 1;
      }
    }
    release();
  }
  void release() {
    for (auto e : ev) hipEventDestroy(e);
    ev.clear();
    cls.clear();
  }
};

static imf_status spectrum_slot(imf_ctx* c, const Plan& p, const std::string& key,
                                SpecEntry** hit, float2** ptr) {
  char buf[64];
  snprintf(buf, sizeof buf, "|%d,%d,%d", p.P[0], p.P[1], p.P[2]);
  const std::string k = key + buf;
  auto it = c->spectra.find(k);
  if (it != c->spectra.end()) {
    it->second.tick = ++c->tick;
    *hit = &it->second;
    *ptr = it->second.ptr;
    return IMF_OK;
  }
  *hit = nullptr;
  *ptr = nullptr;
  const size_t bytes = sizeof(float2) * p.spec_elems;
  if (c->spec_bytes + c->arena_bytes + c->raster_bytes + bytes > c->budget) return IMF_OK;
  float2* q = nullptr;
  if (hipMalloc(&q, bytes) != hipSuccess) {
    hipGetLastError();
    return IMF_OK;
  }
  hipEvent_t ev = nullptr;
  HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  c->spectra[k] = SpecEntry{q, bytes, ++c->tick, ev};
  c->spec_bytes += bytes;
  *ptr = q;
  return IMF_OK;
}

// Work of one request between its launch and its completion.
struct Pending {
  Plan p;
  Timer tm;
  hipStream_t s;
  int nb = 0, flag_cap = 0, hits = 0, misses = 0;
  unsigned int* host = nullptr;  // [0..1] fmax, max_err; [2..] per-batch flag counts
  std::chrono::steady_clock::time_point t_start;
  imf_outputs* out = nullptr;
  double kbytes[16] = {0};  // algorithmic bytes per kernel class
  double kops[16] = {0};    // gathered floats of the minimum filter
  // per orientation: lookups and bytes of the minimum pass over all blocks,
  // scaled by the kept fraction once the bound's list lengths are known
  std::vector<double> mf_ops, mf_bytes;
  int kept_at = -1;         // offset of the kept counts in host[], or -1
  int graph = 0;            // 0 kernel by kernel, 1 captured and launched, 2 replayed
  unsigned long long Fq = 0;  // exact F_max (fixed point) once finished
  bool hint_ok = false;       // the listed bracket held the band of lambda F_max
  bool gover = false;         // the compact gamma stack overflowed: a second pass decides
};

// Enqueue the whole request on stream s (no host synchronization after the
// rasters exist).  The caller holds the context lock.
static imf_status compute_launch(imf_ctx* c, const imf_request* r, const imf_outputs* out,
                                 hipStream_t s, Arena& ar, Pending& pd,
                                 const unsigned long long* known_Fq = nullptr) {
  STCHK(validate(r));
  if (!out) return fail(IMF_EINVAL, "outputs is NULL");
  HIPCHK(hipSetDevice(c->device));
  pd.t_start = std::chrono::steady_clock::now();
  pd.s = s;
  pd.out = const_cast<imf_outputs*>(out);
  std::vector<Orient> os;
  STCHK(enumerate(c, r, os));
  Timer& tm = pd.tm;
  tm.s = s;
  tm.fine = (r->flags & IMF_FLAG_PROFILE) != 0;
  tm.mark(15);
  STCHK(ensure_rasters(c, r, os, s));
  tm.mark(0);
  Plan& p = pd.p;
  STCHK(make_plan(c, r, out, os, p, known_Fq));
  if (out->debug_overlap && (out->debug_orient < 0 || out->debug_orient >= p.nO))
    return fail(IMF_EINVAL, "debug_orient out of range");
  STCHK(arena_reserve(c, ar, p.ws_bytes));
  const long long N = p.N;
  const int h = p.P[0] / 2 + 1;
  const int nb = (int)p.bset.size();
  pd.nb = nb;
  if (nb + 34 > (1 << 14)) return fail(IMF_EINVAL, "too many batches");
  const int nps = std::max(p.nsets, 1);
  // carve the workspace (same order as make_plan)
  float* f = carve<float>(ar, N);
  uint8_t* om = carve<uint8_t>(ar, N);
  const long long ps_stride = (r->nx + 1) * (long long)r->ny * r->nz;
  long long* ps = carve<long long>(ar, ps_stride * nps);
  uint8_t* setfix = p.nsets ? carve<uint8_t>(ar, N * (p.nsets + 1)) : nullptr;
  unsigned int* misc = carve<unsigned int>(ar, 64);
  // misc: [0] float32 max of f over Omega_0, [1] max |g - rint g| (binary),
  // [4] max f at a batch's start, [8..9] skipped pairs, [16..17] F_max in
  // fixed point, [18] candidates of the maximum, [19] band entries, [20] max
  // |g32 - g| of exact recomputations (density), [21] exact recomputations of
  // the post pass, [22] 1 when the expected threshold's bracket held the band,
  // [23] entries of the bracket lists, [24] design voxels outside the value set,
  // [25] the compact gamma stack overflowed, [26..27] its slots taken
  unsigned int* fmax_bits = misc;
  unsigned int* maxerr_bits = misc + 1;
  unsigned long long* Fq = (unsigned long long*)(misc + 16);
  unsigned int* derr_bits = misc + 20;
  int* flag_cnt = carve<int>(ar, nb + 1);
  const int flag_cap = 1 << 20;
  pd.flag_cap = flag_cap;
  int2* flags = carve<int2>(ar, flag_cap);
  imf_orient_desc* d_desc = carve<imf_orient_desc>(ar, (size_t)p.nO * 2);
  imf_orient_desc* d_sweep = d_desc + p.nO;
  // overlaps of one batch, or with gst of every orientation (processing order)
  float* g = carve<float>(ar, (size_t)(p.gst ? p.nO : p.B) * p.max_vol);
  float* lvl = carve<float>(ar, (size_t)p.B * std::max(p.nlvl, 1) * p.max_vol);
  float* gstack = p.gam ? carve<float>(ar, p.gcomp ? (size_t)p.gcap : (size_t)N * p.nO) : nullptr;
  long long* gbase = p.gcomp ? carve<long long>(ar, p.nO) : nullptr;
  int* koff = p.gcomp ? carve<int>(ar, (size_t)p.nO * p.nwords_blk) : nullptr;
  uint64_t* intmask =
      p.intmask ? carve<uint64_t>(ar, (size_t)p.nO * r->nz * r->ny * p.words) : nullptr;
  int* cand = p.exact ? carve<int>(ar, p.cand_cap) : nullptr;
  unsigned long long* cmin = p.exact ? carve<unsigned long long>(ar, p.cand_cap) : nullptr;
  int4* band = p.exact ? carve<int4>(ar, p.band_cap) : nullptr;
  unsigned* bcnt = p.exact ? carve<unsigned>(ar, (size_t)p.nO * IMF_BR_SLICES) : nullptr;
  uint64_t* om_bits = p.exact ? carve<uint64_t>(ar, (size_t)r->nz * r->ny * p.words) : nullptr;
  const int bslot = p.exact ? (int)(p.band_cap / ((long long)p.nO * IMF_BR_SLICES)) : 0;
  unsigned int* cellmin = p.bnb ? carve<unsigned int>(ar, p.B * p.cell_stride) : nullptr;
  // the bound's cell minima come from the inverse x pass (and the recheck)
  // on the transform path, from a pass over g on the direct path
  const bool cm_fused = p.bnb && p.method == IMF_METHOD_FFT;
  int cwx = 1, cwy = 1, cwz = 1;
  imf_block_dims(p.shape, cwx, cwy, cwz);
  int* fpbuf = p.bnb ? carve<int>(ar, p.B * (long long)(kFpCap + 1)) : nullptr;
  float* fblock = p.bnb ? carve<float>(ar, p.nblocks) : nullptr;
  int* wlist = p.bnb ? carve<int>(ar, p.B * p.nblocks) : nullptr;
  int* wcount = p.bnb ? carve<int>(ar, p.B) : nullptr;
  int* kept = p.bnb ? carve<int>(ar, p.nO) : nullptr;
  unsigned long long* wmask = p.bnb ? carve<unsigned long long>(ar, p.B * p.nwords_blk) : nullptr;
  int* woff = p.bnb ? carve<int>(ar, p.B * p.nwords_blk) : nullptr;
  unsigned long long* keepbits =
      p.bnb && p.gam ? carve<unsigned long long>(ar, (size_t)p.nO * p.nwords_blk) : nullptr;
  const long long dc_stride = ((p.max_m[0] + 63) / 64) * (long long)p.max_m[1] * p.max_m[2];
  uint64_t* dc = p.sweep ? carve<uint64_t>(ar, p.B * dc_stride) : nullptr;
  float2 *rho_hat = nullptr, *fw1 = nullptr, *fw2 = nullptr, *tw1 = nullptr, *tw2 = nullptr,
         *bspec = nullptr, *w1 = nullptr, *w2 = nullptr;
  const long long tw1_stride = (long long)p.max_t[2] * p.max_t[1] * h;
  const long long tw2_stride = (long long)p.max_t[2] * p.P[1] * h;
  const long long w1_stride = (long long)p.max_m[2] * p.P[1] * h;
  const long long w2_stride = (long long)p.max_m[2] * p.max_m[1] * h;
  if (p.method == IMF_METHOD_FFT) {
    rho_hat = carve<float2>(ar, p.spec_elems * nps);
    fw1 = carve<float2>(ar, (long long)r->nz * r->ny * h);
    fw2 = carve<float2>(ar, (long long)r->nz * p.P[1] * h);
    tw1 = carve<float2>(ar, p.B * tw1_stride);
    tw2 = carve<float2>(ar, p.B * tw2_stride);
    bspec = carve<float2>(ar, p.B * p.spec_elems);
    w1 = carve<float2>(ar, p.B * w1_stride);
    w2 = carve<float2>(ar, p.B * w2_stride);
  }
  imf_orient_desc* d_miss = nullptr;
  if (p.method == IMF_METHOD_FFT) d_miss = carve<imf_orient_desc>(ar, (size_t)nb * p.B);
  if (ar.used > ar.cap) return fail(IMF_EDEVICE, "workspace layout mismatch");
  // spectra: cached slots (or the batch buffer); wait for cached spectra that
  // another stream may still be writing
  std::vector<char> need_fft(p.nO, 0);
  std::vector<SpecEntry*> fresh(p.nO, nullptr);
  if (p.method == IMF_METHOD_FFT) {
    for (int q = 0; q < p.nO; q++) {
      SpecEntry* hit = nullptr;
      float2* ptr = nullptr;
      if (p.cache) STCHK(spectrum_slot(c, p, p.keys[q], &hit, &ptr));
      if (hit) {
        pd.hits++;
        p.desc[q].spec = ptr;
        HIPCHK(hipStreamWaitEvent(s, hit->ready, 0));
      } else {
        pd.misses++;
        need_fft[q] = 1;
        if (ptr) {
          char buf[64];
          snprintf(buf, sizeof buf, "|%d,%d,%d", p.P[0], p.P[1], p.P[2]);
          fresh[q] = &c->spectra.at(p.keys[q] + buf);
        }
        p.desc[q].spec = ptr ? ptr : bspec + (long long)(q % p.B) * p.spec_elems;
      }
    }
  }
  // Batches whose computed spectra all stay transient (no room in the
  // cache): the tool's z transform is left to the product pass, which reads
  // the tool after its x and y transforms (tdim z planes of them) instead of
  // a whole spectrum written and read back (App. B's pruned transform, fused).
  std::vector<char> fused(nb, 0);
  if (p.method == IMF_METHOD_FFT)
    for (int b = 0; b < nb; b++) {
      int nm = 0;
      bool transient = true;
      for (int q = p.bstart[b]; q < p.bstart[b + 1]; q++)
        if (need_fft[q]) {
          nm++;
          if (fresh[q]) transient = false;
        }
      fused[b] = nm > 0 && transient;
      if (fused[b])
        for (int q = p.bstart[b], m = 0; q < p.bstart[b + 1]; q++)
          if (need_fft[q]) p.desc[q].tmid = tw2 + (long long)(m++) * tw2_stride;
    }
  p.sweep_desc = p.desc;
  for (int q = 0; q < p.nO; q++) {
    p.sweep_desc[q].sruns = p.ent[q]->sxruns;
    p.sweep_desc[q].n_sruns = p.ent[q]->ext[17];
    p.sweep_desc[q].n_sruns1 = 0;
  }
  // descriptors: all of them, and per batch the orientations whose spectra are computed
  std::vector<imf_orient_desc> hall(p.desc);
  hall.insert(hall.end(), p.sweep_desc.begin(), p.sweep_desc.end());
  std::vector<int> nmiss(nb, 0);
  std::vector<imf_orient_desc> hmiss;
  if (d_miss) {
    hmiss.resize((size_t)nb * p.B);
    for (int b = 0; b < nb; b++)
      for (int q = p.bstart[b]; q < p.bstart[b + 1]; q++)
        if (need_fft[q]) hmiss[(size_t)b * p.B + nmiss[b]++] = p.desc[q];
  }
  HIPCHK(hipMemcpy(d_desc, hall.data(), sizeof(imf_orient_desc) * hall.size(),
                   hipMemcpyHostToDevice));
  if (d_miss)
    HIPCHK(hipMemcpy(d_miss, hmiss.data(), sizeof(imf_orient_desc) * hmiss.size(),
                     hipMemcpyHostToDevice));
  const float2 *twx = nullptr, *twy = nullptr, *twz = nullptr;
  if (p.method == IMF_METHOD_FFT) {
    STCHK(get_twiddles(c, p.P[0], &twx));
    STCHK(get_twiddles(c, p.P[1], &twy));
    STCHK(get_twiddles(c, p.P[2], &twz));
  }
  // Everything from here to the statistics copies is stream work only, so it
  // can be captured into a graph: a repeated request with the same signature
  // (request fields, pointers, descriptors, cache state, workspace) replays it.
  const bool graphable = !(r->flags & (IMF_FLAG_NO_GRAPH | IMF_FLAG_PROFILE | IMF_FLAG_PLAIN)) &&
                         pd.misses == 0;
  std::string sig;
  if (graphable) {
    auto put = [&](const void* v, size_t n) { sig.append((const char*)v, n); };
    const long long req_i[] = {r->ndim, r->nx, r->ny, r->nz, r->design_is_density, r->n_tools,
                               r->dir_kind, r->sharp, r->method, r->batch, (long long)r->flags};
    put(req_i, sizeof(req_i));
    const double req_d[] = {r->lambda, r->tau, r->mask_theta_abs};
    put(req_d, sizeof(req_d));
    const void* ptrs[] = {r->design, r->fixture, r->domain, out->imf, out->imf_norm,
                          out->secluded, out->acc_masks, out->debug_overlap};
    put(ptrs, sizeof(ptrs));
    put(&out->debug_orient, sizeof(int));
    long long ndir = 0;
    for (int i = 0; i < r->n_tools; i++) {
      put(&r->tool_ids[i], sizeof(int));
      put(&r->n_dirs[i], sizeof(int));
      ndir += r->n_dirs[i];
    }
    put(r->dirs, (size_t)ndir * r->ndim * (r->dir_kind == IMF_DIR_LATTICE ? 4 : 8));
    put(&r->n_fixture_sets, sizeof(int));
    if (r->n_fixture_sets) {
      put(&r->fixture_sets, sizeof(void*));
      put(r->fixture_of, sizeof(int) * (size_t)ndir);
    }
    put(&p.B, sizeof(p.B));
    put(p.P, sizeof(p.P));
    // launch parameters the autotuner may change after a capture
    const int lp[7] = {p.shape, p.tuned_batch, p.tuned_shape, p.wg_per_cu, c->mf_sync,
                       p.fft_plan, (int)p.defer_appends};
    put(lp, sizeof lp);
    const int sw[3] = {(int)c->lattice_runs, (int)c->spread_order, (int)c->overlap_stack};
    put(sw, sizeof sw);
    // the compact gamma stack's capacity moves every workspace offset after it
    put(&p.gcap, sizeof(p.gcap));
    put(&p.gst, sizeof(p.gst));
    put(&p.known_Fq, sizeof(p.known_Fq));
    put(&p.hinted, sizeof(p.hinted));
    const double br[2] = {p.blo, p.bhi};
    put(br, sizeof br);
    put(&ar.base, sizeof(ar.base));
    put(&ar.host, sizeof(ar.host));
    const void* tws[3] = {twx, twy, twz};
    put(tws, sizeof(tws));
    put(hall.data(), sizeof(imf_orient_desc) * hall.size());
    for (const auto& k : p.keys) sig += k + "|";
  }
  auto launch_all = [&](hipStream_t s) -> imf_status {
  // setup
  HIPCHK(imf_launch_fill_u32(misc, 64, 0u, s));
  HIPCHK(imf_launch_fill_u32((unsigned*)flag_cnt, nb + 1, 0u, s));
  // fixture of each setup (the common fixture with that setup's set) and their union
  const uint8_t* fix_all = r->fixture;
  if (p.nsets) {
    for (int k = 0; k < p.nsets; k++)
      HIPCHK(imf_launch_or_u8(r->fixture, r->fixture_sets + (size_t)N * k, setfix + N * k, N, s));
    uint8_t* uni = setfix + N * p.nsets;
    HIPCHK(imf_launch_or_u8(nullptr, setfix, uni, N, s));
    for (int k = 1; k < p.nsets; k++) HIPCHK(imf_launch_or_u8(uni, setfix + N * k, uni, N, s));
    fix_all = uni;
  }
  HIPCHK(imf_launch_omega0(fix_all, r->domain, om, N, s));
  if (p.hinted) HIPCHK(imf_launch_fill_u32(bcnt, (long long)p.nO * IMF_BR_SLICES, 0u, s));
  HIPCHK(imf_launch_fill_f(f, N, INFINITY, s));
  if (fblock) HIPCHK(imf_launch_fill_f(fblock, p.nblocks, INFINITY, s));
  // the minimum pass writes the mask chunks of the blocks it computes: clear
  // the rest (skipped blocks, and the bits past nx of each row)
  if (p.masks && p.theta_known && !p.sweep)
    HIPCHK(imf_launch_fill_u32((unsigned*)out->acc_masks,
                               2LL * p.nO * r->nz * r->ny * ((r->nx + 63) / 64), 0u, s));
  // blocks the bound skips write no gamma: the mask pass reads their keep bits
  for (int k = 0; k < nps; k++)
    HIPCHK(imf_launch_prefix_x(r->design, r->design_is_density,
                               p.nsets ? setfix + N * k : r->fixture, r->nx, r->ny, r->nz,
                               ps + ps_stride * k, k == 0 ? misc + 24 : nullptr, s));
  tm.mark(1);
  const double esz = r->design_is_density ? 4.0 : 1.0;
  const double S = 8.0 * (double)p.spec_elems;
  const bool has_fix = r->fixture || p.nsets;
  // Omega_0 (fixture read, mask write), f fill, per set the prefix sums
  // (design and fixture read, sums written), per set the fixture and union masks
  pd.kbytes[1] = (double)N * ((has_fix ? 1 : 0) + 1 + 4) +
                 nps * ((double)N * (esz + (has_fix ? 1 : 0)) + 8.0 * ps_stride) +
                 6.0 * N * p.nsets;
  if (p.method == IMF_METHOD_FFT) {
    pd.kbytes[2] = nps * ((double)N * (esz + (has_fix ? 1 : 0)) + S);
    for (int k = 0; k < nps; k++) {
      imf_fwd_design_args fa{r->design, r->design_is_density,
                             p.nsets ? setfix + N * k : r->fixture, r->nx, r->ny, r->nz,
                             p.P[0], p.P[1], p.P[2], fw1, fw2, rho_hat + p.spec_elems * k};
      HIPCHK(imf_launch_fwd_design(fa, p.fl[0], p.fl[1], p.fl[2], twx, twy, twz, s));
    }
    tm.mark(2);
  }
  for (int b = 0; b < nb; b++) {
    const int q0 = p.bstart[b];
    const int nq = p.bstart[b + 1] - q0;
    // the obstacle of this batch's setup: its spectrum and prefix sums
    const long long* ps_b = ps + ps_stride * p.bset[b];
    // this batch's overlaps: its slice of the stack, or the one batch buffer
    float* const gb = p.gst ? g + (size_t)q0 * p.max_vol : g;
    const float2* rho_hat_b = rho_hat ? rho_hat + p.spec_elems * p.bset[b] : nullptr;
    const imf_orient_desc* bd = d_desc + q0;
    // algorithmic bytes of this batch, per kernel class
    for (int q = q0; q < q0 + nq; q++) {
      const imf_orient_desc& d = p.desc[q];
      const double M3 = (double)d.box_dim[0] * d.box_dim[1] * d.box_dim[2];
      if (p.method == IMF_METHOD_FFT) {
        if (need_fft[q]) {
          const double tx = 8.0 * d.tdim[2] * d.tdim[1] * h, ty = 8.0 * d.tdim[2] * p.P[1] * h;
          pd.kbytes[3] += tx + 16.0 * d.n_truns;
          pd.kbytes[4] += tx + ty;
          pd.kbytes[5] += ty + S;
        }
        const double w1b = 8.0 * d.box_dim[2] * p.P[1] * h;
        const double w2b = 8.0 * d.box_dim[2] * d.box_dim[1] * h;
        pd.kbytes[6] += S + w1b;
        pd.kbytes[7] += w1b + w2b;
        pd.kbytes[8] += w2b + 4.0 * M3;
      } else {
        pd.kbytes[8] += 4.0 * M3 + 16.0 * d.n_truns;
      }
      pd.kbytes[10] += 4.0 * M3 * (1 + d.nlvl);
      // lookups: 2 per run and output lane (padding lanes of partial blocks included)
      const double lanes = 64.0 * p.nblocks;
      const double ops = lanes * (2.0 * d.n_sruns - d.n_sruns1);
      // g box read once, runs, f read + write, masks (Omega_0 + bits) or the gamma stack
      const double byt = 4.0 * M3 + 16.0 * d.n_sruns + 8.0 * N +
                         (p.masks && p.theta_known && !p.sweep ? N + N / 8.0 : 0.0) +
                         (p.two_phase ? 4.0 * N : 0.0);
      if (p.bnb) pd.kbytes[15] += 12.0 * p.nblocks;  // block maxima, keep bits, list
      pd.mf_ops.push_back(ops);
      pd.mf_bytes.push_back(byt);
      pd.kops[11] += ops;
      pd.kbytes[11] += byt;
      if (p.sweep) pd.kbytes[12] += 4.0 * M3 + N / 8.0 + N;
    }
    if (p.method == IMF_METHOD_FFT) pd.kbytes[6] += S;  // rho_hat, once per batch
    if (p.method == IMF_METHOD_FFT) {
      if (nmiss[b]) {
        imf_tool_fft_args ta{d_miss + (size_t)b * p.B, nmiss[b], p.P[0], p.P[1], p.P[2],
                             p.max_t[1], p.max_t[2], tw1, tw2, tw1_stride, tw2_stride};
        for (int stage = 0; stage < (fused[b] ? 2 : 3); stage++) {
          HIPCHK(imf_launch_tool_fft(ta, p.fl[1], p.fl[2], twx, twy, twz, s, stage));
          tm.mark(3 + stage);
        }
        for (int q = q0; q < q0 + nq; q++)
          if (fresh[q]) HIPCHK(hipEventRecord(fresh[q]->ready, s));
      }
      imf_inv_args ia{};
      ia.desc = bd;
      ia.nq = nq;
      ia.rho_hat = rho_hat_b;
      ia.px = p.P[0];
      ia.py = p.P[1];
      ia.pz = p.P[2];
      ia.max_mx = p.max_m[0];
      ia.max_my = p.max_m[1];
      ia.max_mz = p.max_m[2];
      ia.w1 = w1;
      ia.w1_stride = w1_stride;
      ia.w2 = w2;
      ia.w2_stride = w2_stride;
      ia.g = gb;
      ia.g_stride = p.max_vol;
      ia.binary = !r->design_is_density;
      ia.delta = 0.25f;
      // density: thresholds known before the request runs, each decided
      // exactly by recomputing the overlaps within E of it (first-pass masks
      // at theta; B at theta_B when lambda = 0 or F_max is given)
      ia.nth = 0;
      if (r->design_is_density) {
        if (p.theta_known) ia.th[ia.nth++] = p.theta;
        if (p.thB_known && !(p.theta_known && p.thB == p.theta)) ia.th[ia.nth++] = p.thB;
      }
      ia.band = p.band;
      ia.max_err_bits = maxerr_bits;
      ia.flag_cnt = flag_cnt + b;
      ia.flag_cap = flag_cap;
      ia.flags = flags;
      if (p.hinted) {
        ia.blist = band;
        ia.bcnt = bcnt;
        ia.bslot = bslot;
        ia.blo = p.blo;
        ia.bhi = p.bhi;
        ia.q0 = q0;
      }
      ia.cellmin = cm_fused ? cellmin : nullptr;
      for (int k = 0; k < 3; k++) ia.fplan[k] = (p.fft_plan >> (2 * k)) & 3;
      ia.fused = fused[b];
      ia.defer = p.defer_appends ? 1 : 0;
      ia.cell_stride = p.cell_stride;
      ia.cwx = cwx;
      ia.cwy = cwy;
      ia.cwz = cwz;
      for (int stage = 0; stage < 3; stage++) {
        HIPCHK(imf_launch_inverse(ia, p.fl[0], p.fl[1], p.fl[2], twx, twy, twz, s, stage));
        tm.mark(6 + stage);
      }
      if (ia.binary || ia.nth) {
        HIPCHK(imf_launch_recheck(bd, ps_b, r->nx, r->ny, r->nz, r->design_is_density, flag_cnt + b,
                                  flags, flag_cap, ia.nth, ia.th[0], ia.th[1], gb, p.max_vol,
                                  ia.cellmin, p.cell_stride, cwx, cwy, cwz, derr_bits, s));
        tm.mark(9);
      }
    } else {
      // exact sums rounded to float32, each known threshold's decision kept
      int nth = 0;
      double th[2] = {0, 0};
      if (r->design_is_density) {
        if (p.theta_known) th[nth++] = p.theta;
        if (p.thB_known && !(p.theta_known && p.thB == p.theta)) th[nth++] = p.thB;
      }
      HIPCHK(imf_launch_direct(bd, nq, ps_b, r->nx, r->ny, r->nz, r->design_is_density, gb,
                               p.max_vol, (int)p.max_vol, nth, th[0], th[1], s));
      tm.mark(8);
    }
    if (out->debug_overlap && p.debug_pos >= q0 && p.debug_pos < q0 + nq) {
      const imf_orient_desc& d = p.desc[p.debug_pos];
      const long long vol = (long long)d.box_dim[0] * d.box_dim[1] * d.box_dim[2];
      HIPCHK(hipMemcpyAsync(out->debug_overlap, gb + (long long)(p.debug_pos - q0) * p.max_vol,
                            sizeof(float) * vol, hipMemcpyDeviceToDevice, s));
      tm.mark(14);
    }
    imf_min_args ma{};
    ma.desc = bd;
    ma.nq = nq;
    ma.g = gb;
    ma.g_stride = p.max_vol;
    ma.lvl = lvl;
    ma.lvl_stride = (long long)std::max(p.nlvl, 1) * p.max_vol;
    ma.nlvl = p.nlvl;
    ma.max_m = 1;
    ma.max_lines = 1;
    ma.stream_waves = 0;
    ma.vstream_waves = 0;
    ma.x_rows = 0;
    ma.lds_levels = 0;
    for (int q = q0; q < q0 + nq; q++) {
      const imf_orient_desc& d = p.desc[q];
      const int ax = d.s_axis;
      if (ax == 3) {  // runs along a lattice vector (at most six levels)
        ma.vstream_waves = std::max(ma.vstream_waves, imf_vlines_of(d.sv, d.box_dim).waves);
        continue;
      }
      ma.max_m = std::max(ma.max_m, d.box_dim[ax]);
      const long long lines =
          ax == 0 ? ((long long)d.box_dim[1] * d.box_dim[2] + 3) / 4
                  : (long long)((d.box_dim[0] + 15) / 16) * (ax == 1 ? d.box_dim[2] : d.box_dim[1]);
      ma.max_lines = std::max(ma.max_lines, lines);
      if (ax != 0)
        ma.stream_waves = std::max(ma.stream_waves, (long long)((d.box_dim[0] + 63) / 64) *
                                                        (ax == 1 ? d.box_dim[2] : d.box_dim[1]));
      else
        ma.x_rows = std::max(ma.x_rows, (long long)d.box_dim[1] * d.box_dim[2]);
      if (d.nlvl > 6) ma.lds_levels = 1;  // beyond the register forms (LS_MAXL)
    }
    ma.nx = r->nx;
    ma.ny = r->ny;
    ma.nz = r->nz;
    ma.f = f;
    ma.omega0 = om;
    ma.masks_on = p.masks && p.theta_known && !p.sweep;
    ma.theta = p.theta;
    ma.masks = out->acc_masks;
    ma.gamma_stack = gstack;
    ma.bnb = p.bnb;
    ma.shape = p.shape;
    ma.cellmin = cellmin;
    ma.cellmin_fused = cm_fused;
    ma.cell_stride = p.cell_stride;
    ma.cell_waves = p.cell_waves;
    ma.fp = fpbuf;
    ma.fp_cap = kFpCap;
    ma.fblock = fblock;
    ma.list = wlist;
    ma.list_stride = p.nblocks;
    ma.count = wcount;
    ma.kept = kept;
    ma.wmask = wmask;
    ma.woff = woff;
    ma.wstride = p.nwords_blk;
    ma.fmax_up = gstack ? misc + 4 : nullptr;
    ma.theta_lambda = r->lambda;
    ma.e_theta = p.E;
    ma.fmargin = p.exact ? 2.0 * p.E : 0.0;
    ma.theta_known = p.theta_known;
    ma.q0 = q0;
    ma.n_cu = c->n_cu;
    ma.wg_per_cu = p.wg_per_cu;
    ma.skipped = (unsigned long long*)(misc + 8);
    ma.sync_waves = c->mf_sync;
    ma.keepbits = keepbits;
    if (p.gcomp) {
      ma.gbase = gbase;
      ma.koff = koff;
      ma.gused = (unsigned long long*)(misc + 26);
      ma.gover = misc + 25;
      ma.gcap = p.gcap;
    }
    HIPCHK(imf_launch_minfilter(ma, s, 0));
    tm.mark(10);
    for (int q = 0; q < nq; q++) {
      if (p.bnb) {
        HIPCHK(imf_launch_minfilter(ma, s, 1, q));
        tm.mark(15);
      }
      HIPCHK(imf_launch_minfilter(ma, s, 2, q));
      tm.mark(11);
    }
    if (p.sweep) {
      imf_sweep_args sa{d_sweep + q0, nq, gb, p.max_vol, p.theta, r->nx, r->ny, r->nz, om, dc,
                        dc_stride, out->acc_masks};
      HIPCHK(imf_launch_sweep(sa, s));
      tm.mark(12);
    }
  }
  // F_max, theta_B = lambda F_max, masks at theta_B, B, fbar, Gamma
  HIPCHK(imf_launch_fmax(f, om, N, fmax_bits, s));
  imf_exact_args ea{};
  ea.desc = d_desc;
  ea.nO = p.nO;
  ea.nx = r->nx;
  ea.ny = r->ny;
  ea.nz = r->nz;
  ea.N = N;
  ea.ps = ps;
  ea.ps_stride = ps_stride;
  ea.f = f;
  ea.omega0 = om;
  ea.gamma = gstack;
  ea.keep = keepbits;
  ea.gbase = gbase;
  ea.koff = koff;
  ea.kstride = p.nwords_blk;
  imf_block_dims(p.shape, ea.WX, ea.WY, ea.WZ);
  ea.gst = p.gst ? g : nullptr;
  ea.gst_stride = p.max_vol;
  ea.E = p.E;
  ea.scale = p.scale;
  ea.lambda = r->lambda;
  ea.fmax_bits = fmax_bits;
  ea.Fq = Fq;
  ea.cand = cand;
  ea.cand_cnt = misc + 18;
  ea.cand_cap = p.cand_cap;
  ea.band = band;
  ea.band_cnt = misc + 19;
  ea.band_cap = p.band_cap;
  ea.err_bits = derr_bits;
  ea.n_exact = misc + 21;
  uint64_t* const mB = p.two_phase ? out->acc_masks : intmask;  // masks at theta_B
  ea.masks = mB;
  // without room for the overlaps (and no expected threshold) the band is
  // decided by a second pass that knows theta_B from this pass's exact F_max:
  // this pass stops at F_max
  const bool second = p.exact && !p.gst && !p.hinted;
  // misc[22]: 1 when the listed bracket holds the band (no scan, no second pass)
  ea.skip_scan = p.hinted ? misc + 22 : nullptr;
  if (p.hinted) {
    ea.blist = band;
    ea.bcnt = bcnt;
    ea.bslot = bslot;
  }
  ea.blisted = misc + 23;
  tm.mark(13);
  if (p.known) {
    HIPCHK(imf_launch_fill_u32(misc + 16, 1, (unsigned)(p.known_Fq & 0xffffffffu), s));
    HIPCHK(imf_launch_fill_u32(misc + 17, 1, (unsigned)(p.known_Fq >> 32), s));
  } else if (p.exact) {
    HIPCHK(imf_launch_exact_fmax(ea, cmin, s));
    if (p.hinted) HIPCHK(imf_launch_bracket_check(ea, p.blo, p.bhi, misc + 22, s));
    tm.mark(9);
  } else {
    HIPCHK(imf_launch_fq_from_fmax(fmax_bits, 1.0 / p.scale, Fq, s));
  }
  if (p.gam && !second && mB) {
    HIPCHK(imf_launch_masks_from_gamma(gstack, p.nO, om, r->nx, r->ny, r->nz, Fq, p.scale,
                                       r->lambda, p.exact ? p.E : 0.0, mB, keepbits, p.shape,
                                       p.nwords_blk, gbase, koff, s));
    tm.mark(13);
  }
  if (p.exact && (p.gst || p.hinted)) {
    // the band: from the listed bracket when it holds it, else from a scan of
    // the stored overlaps (without them a second pass follows)
    if (p.gst) HIPCHK(imf_launch_band_scan(ea, p.max_vol, s));
    HIPCHK(imf_launch_om_bits(om, r->nx, (long long)r->ny * r->nz, om_bits, s));
    ea.om_bits = om_bits;
    HIPCHK(imf_launch_band_exact(ea, s));
    tm.mark(9);
  }
  if (!second)
    HIPCHK(imf_launch_finalize_exact(ea, r->design, r->design_is_density, r->tau,
                                     p.exact ? p.E : 0.0, out->imf, out->imf_norm,
                                     out->secluded, s));
  tm.mark(13);
  pd.kbytes[13] = (double)N * (4 + 1 + esz + (out->imf ? 4 : 0) + (out->imf_norm ? 4 : 0) +
                               (out->secluded ? 1 : 0)) +
                  (p.gam ? (4.0 * N + N / 8.0) * p.nO : 0.0);
  pd.host = ar.host;
  HIPCHK(hipMemcpyAsync(pd.host, misc, 32 * sizeof(unsigned int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(pd.host + 32, flag_cnt, sizeof(int) * nb, hipMemcpyDeviceToHost, s));
  if (kept && 32 + nb + p.nO <= (1 << 14)) {
    pd.kept_at = 32 + nb;
    HIPCHK(hipMemcpyAsync(pd.host + pd.kept_at, kept, sizeof(int) * p.nO, hipMemcpyDeviceToHost,
                          s));
  }
  return IMF_OK;
  };
  if (!graphable) {
    STCHK(launch_all(s));
  } else if (auto it = c->graphs.find(sig); it != c->graphs.end()) {
    tm.off = true;
    HIPCHK(hipGraphLaunch(it->second.exec, s));
    it->second.tick = ++c->graph_tick;
    std::memcpy(pd.kbytes, it->second.kbytes, sizeof pd.kbytes);
    std::memcpy(pd.kops, it->second.kops, sizeof pd.kops);
    pd.mf_ops = it->second.mf_ops;
    pd.mf_bytes = it->second.mf_bytes;
    pd.kept_at = it->second.kept_at;
    pd.host = ar.host;
    pd.graph = 2;
  } else if (++c->graph_seen[sig] < 2) {
    if (c->graph_seen.size() > 1024) c->graph_seen.clear();
    STCHK(launch_all(s));
  } else {
    // second sighting: capture on the private stream, then launch on s
    if (!c->capture) HIPCHK(hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking));
    tm.off = true;
    HIPCHK(hipStreamBeginCapture(c->capture, hipStreamCaptureModeRelaxed));
    const imf_status st = launch_all(c->capture);
    hipGraph_t gr = nullptr;
    const hipError_t e1 = hipStreamEndCapture(c->capture, &gr);
    if (st != IMF_OK) {
      if (gr) hipGraphDestroy(gr);
      return st;
    }
    if (e1 != hipSuccess) return fail(IMF_EDEVICE, "graph capture: %s", hipGetErrorString(e1));
    hipGraphExec_t ex = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    hipGraphDestroy(gr);
    if (e2 != hipSuccess) return fail(IMF_EDEVICE, "graph instantiate: %s", hipGetErrorString(e2));
    if (c->graphs.size() >= 32) {  // least recently used out
      auto lru = c->graphs.begin();
      for (auto i = c->graphs.begin(); i != c->graphs.end(); ++i)
        if (i->second.tick < lru->second.tick) lru = i;
      HIPCHK(hipStreamSynchronize(s));
      hipGraphExecDestroy(lru->second.exec);
      c->graphs.erase(lru);
    }
    auto& ge = c->graphs[sig];
    ge.exec = ex;
    std::memcpy(ge.kbytes, pd.kbytes, sizeof pd.kbytes);
    std::memcpy(ge.kops, pd.kops, sizeof pd.kops);
    ge.mf_ops = pd.mf_ops;
    ge.mf_bytes = pd.mf_bytes;
    ge.kept_at = pd.kept_at;
    ge.tick = ++c->graph_tick;
    c->graph_seen.erase(sig);
    HIPCHK(hipGraphLaunch(ex, s));
    pd.graph = 1;
  }
  if (out->debug_overlap) {
    const imf_orient_desc& d = p.desc[p.debug_pos];
    for (int a = 0; a < 3; a++) {
      pd.out->debug_box[a] = d.box_lo[a];
      pd.out->debug_box[3 + a] = d.box_dim[a];
    }
  }
  return IMF_OK;
}

// Wait for the request and report its statistics (no context lock needed).
static imf_status compute_finish(Pending& pd, imf_stats* st) {
  hipError_t e = hipStreamSynchronize(pd.s);
  if (e != hipSuccess) {
    pd.tm.release();
    return fail(IMF_EDEVICE, "request failed on the device: %s", hipGetErrorString(e));
  }
  const Plan& p = pd.p;
  if (pd.host[24]) {
    pd.tm.release();
    return fail(IMF_EINVAL,
                "%u design voxels lie outside the design's value set ({0, 1} for binary designs, "
                "multiples of 2^-24 in [0, 1] for densities)", pd.host[24]);
  }
  long long total_flags = 0;
  for (int b = 0; b < pd.nb; b++) {
    const int n = (int)pd.host[32 + b];
    if (n > pd.flag_cap) {
      pd.tm.release();
      return fail(IMF_EACCURACY, "guard band of batch %d flagged %d overlaps (capacity %d)", b, n,
                  pd.flag_cap);
    }
    total_flags += n;
  }
  std::memcpy(&pd.Fq, &pd.host[16], 8);
  pd.hint_ok = p.hinted && pd.host[22] == 1u;
  pd.gover = p.gcomp && pd.host[25] != 0u;
  float derr;
  std::memcpy(&derr, &pd.host[20], 4);
  if (p.exact && pd.host[18] > (unsigned)p.cand_cap) {
    pd.tm.release();
    return fail(IMF_EACCURACY,
                "%u voxels have f within 2E of the float32 maximum (capacity %d): F_max cannot "
                "be decided exactly", pd.host[18], p.cand_cap);
  }
  if (p.exact && pd.host[19] > (unsigned)p.band_cap) {
    pd.tm.release();
    return fail(IMF_EACCURACY, "%u overlaps lie within E of lambda F_max (capacity %d)",
                pd.host[19], p.band_cap);
  }
  // the error model: every exact recomputation must lie well inside the band
  if (p.E > 0 && (double)derr > 0.5 * p.E) {
    pd.tm.release();
    return fail(IMF_EACCURACY,
                "a float32 overlap is %.3g from its exact value, more than half the guard band "
                "E = %.3g: the error model does not hold for this request", (double)derr, p.E);
  }
  if (st) {
    std::memset(st, 0, sizeof *st);
    st->F_max = (double)pd.Fq * p.scale;
    float me;
    std::memcpy(&me, &pd.host[1], 4);
    st->max_frac_err = me;
    st->max_abs_err = derr;
    st->post_exact = pd.host[21];
    st->band_entries = pd.hint_ok ? pd.host[23] : pd.host[19];
    st->guard_flags = total_flags + pd.host[21];
    st->passes = 1;
    st->hinted = p.hinted ? (pd.hint_ok ? 1 : pd.host[22] == 2u ? 3 : 2) : 0;
    if (p.bnb) {
      unsigned long long sk;
      std::memcpy(&sk, &pd.host[8], 8);
      st->bound_skipped = (long long)sk;
      st->bound_blocks = p.nblocks * p.nO;
    }
    st->guard_band = p.E;
    pd.tm.collect(st);
    if (pd.tm.fine) {
      if (pd.kept_at >= 0 && p.nblocks > 0) {  // the minimum pass ran on the kept blocks only
        pd.kops[11] = pd.kbytes[11] = 0;
        for (size_t q = 0; q < pd.mf_ops.size(); q++) {
          const double fr = (double)(int)pd.host[pd.kept_at + q] / (double)p.nblocks;
          pd.kops[11] += fr * pd.mf_ops[q];
          pd.kbytes[11] += fr * pd.mf_bytes[q];
        }
      }
      for (int k = 0; k < 16; k++) {
        st->k_bytes[k] = pd.kbytes[k];
        st->k_ops[k] = pd.kops[k];
      }
    }
    st->t_ms[7] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                            pd.t_start).count();
    st->model_bytes = model_bytes(p);
    for (int a = 0; a < 3; a++) st->P[a] = p.P[a];
    st->n_orient = p.nO;
    st->method = p.method;
    st->batch = p.B;
    st->cache_hits = pd.hits;
    st->cache_misses = pd.misses;
    st->graph = pd.graph;
    for (int q = 0; q < p.nO; q++) {
      st->lattice_runs += p.desc[q].s_axis == 3;
      st->box_voxels += (double)p.desc[q].box_dim[0] * p.desc[q].box_dim[1] * p.desc[q].box_dim[2];
    }
    st->mf_shape = p.shape;
    st->mf_wg_per_cu = p.wg_per_cu;
    st->fft_plan = p.fft_plan;
  } else {
    pd.tm.release();
  }
  return IMF_OK;
}

// Launch and wait for one request.  A density request at lambda F_max whose
// overlaps had no room to stay in the workspace ends its first pass at the
// exact F_max; a second pass then runs with theta_B = lambda F_max known, so
// its first-pass recheck decides the masks and B exactly.  The context lock is
// taken while a pass is planned and launched (recursively when the caller
// holds it), not while it runs.
static imf_status run_request(imf_ctx* c, const imf_request* r, const imf_outputs* out,
                              imf_stats* st, hipStream_t s, Arena& ar) {
  unsigned long long known = 0;
  double t_first = 0;
  long long flags_first = 0;
  int hinted_first = 0;
  double lock_ms = 0, hold_ms = 0;  // waiting for the context lock, holding it
  using clk = std::chrono::steady_clock;
  for (int pass = 0; pass < 2; pass++) {
    Pending pd;
    imf_status e;
    {
      const auto t0 = clk::now();
      std::lock_guard<std::recursive_mutex> lk(c->mu);
      const auto t1 = clk::now();
      e = compute_launch(c, r, out, s, ar, pd, pass ? &known : nullptr);
      lock_ms += std::chrono::duration<double, std::milli>(t1 - t0).count();
      hold_ms += std::chrono::duration<double, std::milli>(clk::now() - t1).count();
      if (e != IMF_OK) {
        hipStreamSynchronize(s);
        pd.tm.release();
        return e;
      }
    }
    imf_stats tmp{};
    e = compute_finish(pd, st ? st : &tmp);
    if (e != IMF_OK) return e;
    if (st) {
      st->lock_ms = lock_ms;
      st->hold_ms = hold_ms;
    }
    if (!pd.p.gkey.empty() && pd.kept_at >= 0 && pd.p.nblocks > 0) {
      // the kept fraction sizes the next compact gamma stack of this shape
      double kept = 0;
      for (int q = 0; q < pd.p.nO; q++) kept += (double)(int)pd.host[pd.kept_at + q];
      std::lock_guard<std::recursive_mutex> lk(c->mu);
      c->gkept[pd.p.gkey] = kept / ((double)pd.p.nO * (double)pd.p.nblocks);
      if (c->gkept.size() > 4096) c->gkept.clear();
    }
    if (pd.p.exact && !pd.p.hint_key.empty()) {
      // remember the exact F_max; a bracket that missed widens next time
      std::lock_guard<std::recursive_mutex> lk(c->mu);
      imf_ctx::Hint h;
      auto old = c->hints.find(pd.p.hint_key);
      if (old != c->hints.end()) {
        h.F[1] = old->second.F[0];
        h.F[2] = old->second.F[1];
      }
      h.F[0] = pd.Fq;
      h.listed = pd.p.hinted ? (double)pd.host[23] / std::max(pd.p.nO, 1) : 0.0;
      // next half-width: 2.5 times this prediction's relative error, decaying
      // by 15% per request, within [0.05%, 6%].  A miss costs a second pass
      // (about the whole request again) and the width only its listed
      // entries, so the width follows the error up quickly and comes down
      // slowly: on a 50-iteration TO loop whose maximum moved by up to 5% a
      // step this missed 2 times where doubling and halving missed 11.
      double err = 0;
      if (pd.p.hinted && pd.Fq > 0)
        err = std::fabs((double)pd.Fq - pd.p.hint_pred) / (double)pd.Fq;
      const double prev = old != c->hints.end() ? old->second.delta : 0.0;
      h.delta = std::min(0.06, std::max(0.0005, std::max(0.85 * prev, 2.5 * err)));
      c->hints[pd.p.hint_key] = h;
      if (c->hints.size() > 4096) c->hints.clear();
    }
    // a second pass with the threshold known: the band of lambda F_max was
    // neither stored nor listed, or the compact gamma stack overflowed
    if (!((pd.p.exact && !pd.p.gst && !pd.hint_ok) || pd.gover)) {
      if (st && pass) {
        st->passes = 2;
        st->t_ms[7] += t_first;
        st->guard_flags += flags_first;
        st->hinted = hinted_first;
      }
      return IMF_OK;
    }
    known = pd.Fq;
    if (st) {
      t_first = st->t_ms[7];
      flags_first = st->guard_flags;
      hinted_first = st->hinted;
    }
  }
  return fail(IMF_EDEVICE, "second pass did not settle the threshold");
}

static imf_status compute_impl(imf_ctx* c, const imf_request* r, const imf_outputs* out,
                               imf_stats* st, hipStream_t s, Arena& ar) {
  return run_request(c, r, out, st, s, ar);
}

extern "C" imf_status imf_compute(imf_ctx* c, const imf_request* r, const imf_outputs* out,
                                  imf_stats* st, void* stream) {
  if (!c) return fail(IMF_EINVAL, "ctx is NULL");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  return compute_impl(c, r, out, st, (hipStream_t)stream, c->arena);
}

// ---------------------------------------------------------------------------
// single steps
// ---------------------------------------------------------------------------
extern "C" imf_status imf_raster(imf_ctx* c, int ndim, const imf_tool* tool, int dir_kind,
                                 const void* dir, int sharp, int32_t* offsets, uint8_t* flags_out,
                                 long long cap, long long* count) {
  if (!c || !tool || !dir || !count) return fail(IMF_EINVAL, "NULL argument");
  if (tool->kind == IMF_TOOL_VOXEL)
    return fail(IMF_EINVAL, "voxel tools are registered first (imf_raster_tool)");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  int tid;
  STCHK(imf_tool_register(c, tool, &tid));
  return imf_raster_tool(c, tid, ndim, dir_kind, dir, sharp, offsets, flags_out, cap, count);
}

extern "C" imf_status imf_raster_tool(imf_ctx* c, int tid, int ndim, int dir_kind,
                                      const void* dir, int sharp, int32_t* offsets,
                                      uint8_t* flags_out, long long cap, long long* count) {
  if (!c || !dir || !count) return fail(IMF_EINVAL, "NULL argument");
  if (ndim != 2 && ndim != 3) return fail(IMF_EINVAL, "ndim must be 2 or 3");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  HIPCHK(hipSetDevice(c->device));
  imf_request r{};
  r.ndim = ndim;
  r.n_tools = 1;
  r.tool_ids = &tid;
  int one = 1;
  r.n_dirs = &one;
  r.dir_kind = dir_kind;
  r.dirs = dir;
  r.sharp = sharp;
  std::vector<Orient> os;
  STCHK(enumerate(c, &r, os));
  imf_raster_desc hd;
  raster_desc_for(c, tid, os[0], ndim, dir_kind == IMF_DIR_LATTICE, sharp, hd);
  const long long vol = (long long)hd.dim[0] * hd.dim[1] * hd.dim[2];
  hd.flags_off = 0;
  hd.rows_off = 0;
  imf_raster_desc* dd = nullptr;
  uint8_t* fl = nullptr;
  int* ext = nullptr;
  HIPCHK(hipMalloc(&dd, sizeof hd));
  HIPCHK(hipMalloc(&fl, (vol + 3) & ~3LL));
  HIPCHK(hipMalloc(&ext, sizeof(int) * IMF_EXT_INTS));
  std::vector<int> hext(IMF_EXT_INTS, 0);
  for (int a = 0; a < 3; a++) {
    hext[a] = hext[6 + a] = 1 << 29;
    hext[3 + a] = hext[9 + a] = -(1 << 29);
  }
  hipStream_t s = c->internal;
  std::vector<uint8_t> hf(vol);
  hipError_t e = hipMemcpyAsync(dd, &hd, sizeof hd, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ext, hext.data(), sizeof(int) * IMF_EXT_INTS, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = imf_launch_raster(dd, 1, (int)vol, fl, ext, s);
  if (e == hipSuccess) e = imf_launch_sharp_subset(dd, 1, (int)vol, fl, ext, s);
  if (e == hipSuccess) e = hipMemcpyAsync(hf.data(), fl, vol, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipFree(dd);
  hipFree(fl);
  hipFree(ext);
  if (e != hipSuccess) return fail(IMF_EDEVICE, "raster: %s", hipGetErrorString(e));
  long long n = 0;
  for (long long i = 0; i < vol; i++) {
    if (!(hf[i] & 5)) continue;
    if (n < cap) {
      const int x = (int)(i % hd.dim[0]), y = (int)((i / hd.dim[0]) % hd.dim[1]),
                z = (int)(i / ((long long)hd.dim[0] * hd.dim[1]));
      if (offsets) {
        offsets[3 * n] = x + hd.lo[0];
        offsets[3 * n + 1] = y + hd.lo[1];
        offsets[3 * n + 2] = z + hd.lo[2];
      }
      if (flags_out) flags_out[n] = hf[i];
    }
    n++;
  }
  *count = n;
  if (n > cap) return fail(IMF_EINVAL, "capacity %lld < %lld voxels", cap, n);
  return IMF_OK;
}

extern "C" imf_status imf_fft_c2c(imf_ctx* c, int n, int batch, const float* in, float* out,
                                  int inverse, void* stream) {
  if (!c || !in || !out) return fail(IMF_EINVAL, "NULL argument");
  imf_fft_len L = make_len(n);
  if (n < 1 || n > 1024 || L.nstages < 0) return fail(IMF_EINVAL, "unsupported length %d", n);
  if (batch < 1) return fail(IMF_EINVAL, "batch must be >= 1");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  HIPCHK(hipSetDevice(c->device));
  const float2* tw;
  STCHK(get_twiddles(c, n, &tw));
  // columns are the batch index (stride 1), elements j at j * batch
  HIPCHK(imf_launch_columns((const float2*)in, (float2*)out, batch, batch, L, tw, inverse,
                            (hipStream_t)stream));
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  return IMF_OK;
}

extern "C" imf_status imf_fft_r2c_3d(imf_ctx* c, int nx, int ny, int nz, int px, int py, int pz,
                                     const float* in, float* out, void* stream) {
  if (!c || !in || !out) return fail(IMF_EINVAL, "NULL argument");
  const imf_fft_len fx = make_len(px), fy = make_len(py), fz = make_len(pz);
  if (fx.nstages < 0 || fy.nstages < 0 || fz.nstages < 0 || px % 2 || px > 1024 || py > 1024 ||
      pz > 1024)
    return fail(IMF_EINVAL, "unsupported transform sizes");
  if (nx > px || ny > py || nz > pz || nx < 1 || ny < 1 || nz < 1)
    return fail(IMF_EINVAL, "grid larger than the transform");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  HIPCHK(hipSetDevice(c->device));
  const float2 *twx, *twy, *twz;
  STCHK(get_twiddles(c, px, &twx));
  STCHK(get_twiddles(c, py, &twy));
  STCHK(get_twiddles(c, pz, &twz));
  const int h = px / 2 + 1;
  float2 *w1 = nullptr, *w2 = nullptr;
  HIPCHK(hipMalloc(&w1, sizeof(float2) * (size_t)nz * ny * h));
  HIPCHK(hipMalloc(&w2, sizeof(float2) * (size_t)nz * py * h));
  imf_fwd_design_args a{in, 1, nullptr, nx, ny, nz, px, py, pz, w1, w2, (float2*)out};
  hipError_t e = imf_launch_fwd_design(a, fx, fy, fz, twx, twy, twz, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  hipFree(w1);
  hipFree(w2);
  if (e != hipSuccess) return fail(IMF_EDEVICE, "fft: %s", hipGetErrorString(e));
  return IMF_OK;
}

// ---------------------------------------------------------------------------
// autotune: time batch widths on a real request and keep the fastest
// ---------------------------------------------------------------------------
extern "C" imf_status imf_heaviside(imf_ctx* c, long long n, const float* xi, double beta,
                                    float* rho, void* stream) {
  if (!c || (n > 0 && (!xi || !rho))) return fail(IMF_EINVAL, "NULL argument");
  if (n < 0 || !std::isfinite(beta) || beta < 0) return fail(IMF_EINVAL, "n >= 0 and beta >= 0");
  if (n == 0) return IMF_OK;
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(imf_launch_heaviside(xi, n, beta, rho, (hipStream_t)stream));
  return IMF_OK;
}

extern "C" imf_status imf_access_filter(imf_ctx* c, int nx, int ny, int nz, const void* design,
                                        int design_is_density, const uint8_t* fixture,
                                        const uint8_t* domain, const float* imf_norm,
                                        const uint8_t* secluded, double tau,
                                        const float* sens_phi, double w_acc, float* filter_out,
                                        float* sens_out, void* stream) {
  if (!c || !design || !imf_norm || !secluded || !filter_out)
    return fail(IMF_EINVAL, "NULL argument");
  if (nx <= 0 || ny <= 0 || nz <= 0) return fail(IMF_EINVAL, "grid sizes must be positive");
  if (sens_phi && (!sens_out || !(w_acc >= 0 && w_acc <= 1)))
    return fail(IMF_EINVAL, "sens_out is NULL or w_acc outside [0, 1]");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  HIPCHK(hipSetDevice(c->device));
  if (!c->couple_scratch) HIPCHK(hipMalloc(&c->couple_scratch, 256));
  imf_couple_args a{};
  a.n = (long long)nx * ny * nz;
  a.design = design;
  a.density = design_is_density;
  a.fixture = fixture;
  a.domain = domain;
  a.imf_norm = imf_norm;
  a.secluded = secluded;
  a.tau = tau;
  a.filt = filter_out;
  a.sens = sens_phi;
  a.w = w_acc;
  a.sens_out = sens_out;
  a.smax = c->couple_scratch;
  HIPCHK(imf_launch_access_filter(a, (hipStream_t)stream));
  return IMF_OK;
}

extern "C" imf_status imf_plan_greedy(imf_ctx* c, int nx, int ny, int nz, int n_orient,
                                      const uint64_t* acc_masks, const void* design,
                                      int design_is_density, const uint8_t* fixture,
                                      const uint8_t* domain, double tau, int max_steps,
                                      int* orient_out, long long* removed_out, int* n_steps,
                                      long long* remaining, void* stream) {
  if (!c || !acc_masks || !design || !n_steps || !remaining ||
      (max_steps > 0 && (!orient_out || !removed_out)))
    return fail(IMF_EINVAL, "NULL argument");
  if (nx <= 0 || ny <= 0 || nz <= 0 || n_orient <= 0 || max_steps < 0)
    return fail(IMF_EINVAL, "sizes must be positive");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  HIPCHK(hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  const long long nw = (long long)nz * ny * ((nx + 63) / 64);
  uint64_t* R = nullptr;
  unsigned long long* counts = nullptr;
  HIPCHK(hipMalloc(&R, sizeof(uint64_t) * nw));
  if (hipMalloc(&counts, sizeof(unsigned long long) * (n_orient + 1)) != hipSuccess) {
    hipFree(R);
    return fail(IMF_ENOMEM, "plan scratch");
  }
  std::vector<unsigned long long> h(n_orient + 1);
  imf_status st = IMF_OK;
  auto run = [&]() -> imf_status {
    HIPCHK(imf_launch_negative_bits(design, design_is_density, tau, fixture, domain, nx,
                                    (long long)ny * nz, R, s));
    int k = 0;
    for (; k < max_steps; k++) {
      HIPCHK(imf_launch_cover_count(acc_masks, n_orient, nw, R, counts, s));
      HIPCHK(hipMemcpyAsync(h.data(), counts, sizeof(unsigned long long) * n_orient,
                            hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      int best = 0;
      for (int q = 1; q < n_orient; q++)
        if (h[q] > h[best]) best = q;
      if (h[best] == 0) break;
      orient_out[k] = best;
      removed_out[k] = (long long)h[best];
      HIPCHK(imf_launch_cover_remove(acc_masks + (long long)best * nw, nw, R, s));
    }
    *n_steps = k;
    // what is left: popcount of R (counted against an all-ones "mask" = R itself)
    HIPCHK(imf_launch_cover_count(R, 1, nw, R, counts, s));
    HIPCHK(hipMemcpyAsync(h.data(), counts, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *remaining = (long long)h[0];
    return IMF_OK;
  };
  st = run();
  hipStreamSynchronize(s);
  hipFree(R);
  hipFree(counts);
  return st;
}

// The same plan without any allocation: scratch in the library's fixed
// per-device array, the step's choice made on the device and read as two
// words into host stack memory.
extern "C" imf_status imf_plan_greedy_noalloc(imf_ctx* c, int nx, int ny, int nz, int n_orient,
                                              const uint64_t* acc_masks, const void* design,
                                              int design_is_density, const uint8_t* fixture,
                                              const uint8_t* domain, double tau, int max_steps,
                                              int* orient_out, long long* removed_out,
                                              int* n_steps, long long* remaining, void* stream) {
  if (!c || !acc_masks || !design || !n_steps || !remaining ||
      (max_steps > 0 && (!orient_out || !removed_out)))
    return fail(IMF_EINVAL, "NULL argument");
  if (nx <= 0 || ny <= 0 || nz <= 0 || n_orient <= 0 || max_steps < 0)
    return fail(IMF_EINVAL, "sizes must be positive");
  const long long nw = (long long)nz * ny * ((nx + 63) / 64);
  const long long need = nw + n_orient + 2;
  if (need > IMF_PLAN_SCRATCH_WORDS)
    return fail(IMF_EINVAL,
                "plan needs %lld scratch words (%lld mask words + %d counts + 2), more than "
                "the %d of the allocation-free planner",
                need, nw, n_orient, IMF_PLAN_SCRATCH_WORDS);
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  HIPCHK(hipSetDevice(c->device));
  unsigned long long* base = imf_plan_scratch(c->device);
  if (!base) return fail(IMF_EDEVICE, "planner scratch not set up on device %d", c->device);
  hipStream_t s = (hipStream_t)stream;
  uint64_t* R = (uint64_t*)base;
  unsigned long long* counts = base + nw;
  unsigned long long* best = counts + n_orient;
  unsigned long long h[2] = {0, 0};
  HIPCHK(imf_launch_negative_bits(design, design_is_density, tau, fixture, domain, nx,
                                  (long long)ny * nz, R, s));
  int k = 0;
  for (; k < max_steps; k++) {
    HIPCHK(imf_launch_cover_count(acc_masks, n_orient, nw, R, counts, s));
    HIPCHK(imf_launch_cover_best(counts, n_orient, best, s));
    HIPCHK(hipMemcpyAsync(h, best, sizeof h, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h[0] == 0) break;
    orient_out[k] = (int)h[1];
    removed_out[k] = (long long)h[0];
    HIPCHK(imf_launch_cover_remove(acc_masks + (long long)h[1] * nw, nw, R, s));
  }
  *n_steps = k;
  HIPCHK(imf_launch_cover_count(R, 1, nw, R, counts, s));
  HIPCHK(hipMemcpyAsync(h, counts, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *remaining = (long long)h[0];
  return IMF_OK;
}

extern "C" imf_status imf_autotune(imf_ctx* c, const imf_request* r, const imf_outputs* out,
                                   int* best_batch) {
  if (!c || !r || !out) return fail(IMF_EINVAL, "NULL argument");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  Plan p0;
  std::vector<Orient> os;
  STCHK(enumerate(c, r, os));
  STCHK(ensure_rasters(c, r, os, c->internal));
  STCHK(make_plan(c, r, out, os, p0));
  // time one candidate: a warm-up request (fills the spectrum cache), then the
  // faster of two timed ones, kernel by kernel
  auto time_one = [&](int B, int shape, int wg, int fft, double& ms) -> imf_status {
    imf_request rr = *r;
    rr.batch = B;
    rr.flags |= IMF_FLAG_NO_GRAPH;
    rr.flags &= ~(unsigned)IMF_FLAG_PROFILE;
    c->force_shape = shape;
    c->force_wg = wg;
    c->force_fft = fft;
    imf_stats st;
    ms = 1e300;
    imf_status s1 = IMF_OK;
    for (int k = 0; k < 3 && s1 == IMF_OK; k++) {
      s1 = compute_impl(c, &rr, out, &st, c->internal, c->arena);
      if (k > 0 && s1 == IMF_OK) ms = std::min(ms, st.t_ms[7]);
    }
    c->force_shape = -1;
    c->force_wg = 0;
    c->force_fft = -1;
    return s1;
  };
  imf_ctx::Tuned best;
  best.shape = p0.tuned_shape;
  best.wg = p0.wg_per_cu;
  best.fft = p0.fft_plan;
  double best_ms = 1e300;
  // batch width with the current tile shapes
  for (int B : {1, 2, 4, 8, 12, 16}) {
    if (B > p0.nO && B != 1) break;
    double ms;
    const imf_status s1 = time_one(B, best.shape, best.wg, best.fft, ms);
    if (s1 == IMF_ENOMEM) break;
    STCHK(s1);
    if (ms < best_ms) {
      best_ms = ms;
      best.batch = B;
    }
  }
  // block shape and resident grid of the sharp-point minimum (3D only); an
  // alternative must win by 2% (timings of near-equal settings flip with
  // noise, and a stable choice keeps profiles of one setting comparable)
  if (p0.nd == 3)
    for (int shape : {2, 4, 0, 1, 3})
      for (int wg : {4, 6, 8}) {
        if (shape == best.shape && wg == best.wg) continue;
        double ms;
        STCHK(time_one(best.batch, shape, wg, best.fft, ms));
        if (ms < 0.98 * best_ms) {
          best_ms = ms;
          best.shape = shape;
          best.wg = wg;
        }
      }
  // transform plan of each inverse pass (radix split, tile width), one pass
  // at a time with the others held (FFT method only); the same 2% margin
  if (p0.method == IMF_METHOD_FFT)
    for (int pass = 0; pass < 3; pass++)
      for (int v = 0; v < 4 && imf_fft_plan_variants(p0.P[2 - pass]); v++) {
        const int cand = (best.fft & ~(3 << (2 * pass))) | (v << (2 * pass));
        if (cand == best.fft) continue;
        double ms;
        STCHK(time_one(best.batch, best.shape, best.wg, cand, ms));
        if (ms < 0.98 * best_ms) {
          best_ms = ms;
          best.fft = cand;
        }
      }
  c->tuned[tune_key(p0)] = best;
  // requests captured before the tuning keep replaying their old launch
  // parameters: drop the captured graphs
  for (auto& kv : c->graphs)
    if (kv.second.exec) hipGraphExecDestroy(kv.second.exec);
  c->graphs.clear();
  c->graph_seen.clear();
  if (best_batch) *best_batch = best.batch;
  return IMF_OK;
}

// The autotuned table as text: a header line, then one line per request shape
// "<method>|<nx>,<ny>,<nz>|<px>,<py>,<pz> <batch> <shape> <wg> <fft>" (version
// 1 tables, without <fft>, load with the default transform plans).
extern "C" imf_status imf_autotune_save(imf_ctx* c, const char* path) {
  if (!c || !path) return fail(IMF_EINVAL, "NULL argument");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(IMF_EINVAL, "cannot write %s", path);
  bool ok = std::fprintf(f, "imf-autotune 2\n") > 0;
  for (const auto& kv : c->tuned)
    ok = ok && std::fprintf(f, "%s %d %d %d %d\n", kv.first.c_str(), kv.second.batch,
                            kv.second.shape, kv.second.wg, kv.second.fft) > 0;
  ok = (std::fclose(f) == 0) && ok;
  return ok ? IMF_OK : fail(IMF_EINVAL, "writing %s failed", path);
}

extern "C" imf_status imf_autotune_load(imf_ctx* c, const char* path, int* n_loaded) {
  if (!c || !path) return fail(IMF_EINVAL, "NULL argument");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(IMF_EINVAL, "cannot read %s", path);
  std::map<std::string, imf_ctx::Tuned> got;
  char line[256];
  int ln = 0, version = 0;
  imf_status st = IMF_OK;
  while (st == IMF_OK && std::fgets(line, sizeof line, f)) {
    ln++;
    if (ln == 1) {
      if (std::strncmp(line, "imf-autotune 1", 14) == 0 && (line[14] == '\n' || !line[14]))
        version = 1;
      else if (std::strncmp(line, "imf-autotune 2", 14) == 0 && (line[14] == '\n' || !line[14]))
        version = 2;
      else
        st = fail(IMF_EINVAL, "%s: not an autotune table", path);
      continue;
    }
    char key[128];
    int m, n[3], P[3], batch, shape, wg, fft = 0, used = 0;
    const int nf = version == 1
                       ? std::sscanf(line, "%127s %d %d %d %n", key, &batch, &shape, &wg, &used)
                       : std::sscanf(line, "%127s %d %d %d %d %n", key, &batch, &shape, &wg,
                                     &fft, &used);
    if (nf != (version == 1 ? 4 : 5) || line[used] != '\0' ||
        std::sscanf(key, "%d|%d,%d,%d|%d,%d,%d", &m, &n[0], &n[1], &n[2], &P[0], &P[1], &P[2]) !=
            7 ||
        batch < 1 || batch > 64 || shape < -1 || shape > 4 || wg < 0 || wg > 16 || fft < 0 ||
        fft > 63) {
      st = fail(IMF_EINVAL, "%s:%d: malformed autotune entry", path, ln);
      break;
    }
    imf_ctx::Tuned t;
    t.batch = batch;
    t.shape = shape;
    t.wg = wg;
    t.fft = fft;
    got[key] = t;
  }
  std::fclose(f);
  if (st == IMF_OK && ln == 0) st = fail(IMF_EINVAL, "%s: empty", path);
  if (st != IMF_OK) return st;
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  for (const auto& kv : got) c->tuned[kv.first] = kv.second;
  if (n_loaded) *n_loaded = (int)got.size();
  return IMF_OK;
}

// ---------------------------------------------------------------------------
// serving: a queue of requests, admitted by workspace footprint, each run on
// a worker with its own stream and workspace (continuous batching: a request
// starts as soon as a worker and memory are free)
// ---------------------------------------------------------------------------
struct Request {
  uint64_t ticket;
  imf_request req;
  imf_outputs out;
  std::vector<int> tool_ids, n_dirs, fixture_of;
  std::vector<char> dirs;
  size_t footprint = 0;
  int bypassed = 0;  // times a later request was admitted ahead of this one
  int state = 0;  // 0 queued, 1 running, 2 done, 3 cancelled
  imf_status status = IMF_OK;
  std::string err;
  imf_stats stats{};
  std::chrono::steady_clock::time_point t_submit;
};

// Admission: the queue's head when its workspace fits beside the running
// requests (half the budget for all of them; a request always fits an idle
// context), else the first of the next kBypassScan requests that fits.  A
// head passed over kMaxBypass times blocks the queue until it fits, so a large
// request waits for memory at most that many admissions.
static const int kBypassScan = 8, kMaxBypass = 4;
static std::deque<std::shared_ptr<Request>>::iterator serve_pick(imf_ctx* c) {
  auto fits = [&](const Request& r) {
    return c->inflight_bytes + r.footprint <= c->budget / 2 || c->n_running == 0;
  };
  if (c->queue.empty()) return c->queue.end();
  auto head = c->queue.begin();
  if (fits(**head)) return head;
  if ((*head)->bypassed >= kMaxBypass) return c->queue.end();
  int k = 0;
  for (auto it = std::next(head); it != c->queue.end() && k < kBypassScan; ++it, ++k)
    if (fits(**it)) return it;
  return c->queue.end();
}

static void serve_worker(imf_ctx* c) {
  hipSetDevice(c->device);
  hipStream_t s;
  hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  Arena ar;
  ar.worker = true;
  for (;;) {
    std::shared_ptr<Request> rq;
    double queued_ms = 0;
    {
      std::unique_lock<std::mutex> lk(c->smu);
      auto pick = c->queue.end();
      c->scv.wait(lk, [&] {
        if (c->stop) return true;
        pick = serve_pick(c);
        return pick != c->queue.end();
      });
      if (c->stop) break;
      rq = *pick;
      if (pick != c->queue.begin()) c->queue.front()->bypassed++;
      c->queue.erase(pick);
      rq->state = 1;
      queued_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                             rq->t_submit)
                      .count();
      c->inflight_bytes += rq->footprint;
      c->n_running++;
    }
    imf_status st;
    {
      // planning and caches are shared: hold the context lock while the
      // request is planned and launched, then wait without it, so kernels of
      // different workers overlap on the device through their streams
      st = run_request(c, &rq->req, &rq->out, &rq->stats, s, ar);
    }
    {
      std::lock_guard<std::mutex> lk(c->smu);
      rq->status = st;
      if (st != IMF_OK) rq->err = g_err;
      rq->stats.t_ms[7] = std::chrono::duration<double, std::milli>(
                              std::chrono::steady_clock::now() - rq->t_submit)
                              .count();
      rq->stats.queue_ms = queued_ms;
      rq->state = 2;
      c->inflight_bytes -= rq->footprint;
      c->n_running--;
    }
    c->scv.notify_all();
  }
  hipStreamSynchronize(s);
  if (ar.base) {
    hipFree(ar.base);
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->arena_bytes -= ar.cap;
  }
  if (ar.host) hipHostFree(ar.host);
  hipStreamDestroy(s);
}

static void serve_shutdown(imf_ctx* c) {
  {
    std::lock_guard<std::mutex> lk(c->smu);
    c->stop = true;
  }
  c->scv.notify_all();
  for (auto& t : c->workers) t.join();
  c->workers.clear();
}

extern "C" imf_status imf_submit(imf_ctx* c, const imf_request* r, const imf_outputs* out,
                                 uint64_t* ticket) {
  if (!c || !r || !out || !ticket) return fail(IMF_EINVAL, "NULL argument");
  STCHK(validate(r));
  auto rq = std::make_shared<Request>();
  rq->req = *r;
  rq->out = *out;
  rq->tool_ids.assign(r->tool_ids, r->tool_ids + r->n_tools);
  rq->n_dirs.assign(r->n_dirs, r->n_dirs + r->n_tools);
  long long nd = 0;
  for (int i = 0; i < r->n_tools; i++) nd += r->n_dirs[i];
  const size_t esz = r->dir_kind == IMF_DIR_LATTICE ? sizeof(int32_t) : sizeof(double);
  rq->dirs.assign((const char*)r->dirs, (const char*)r->dirs + nd * r->ndim * esz);
  rq->req.tool_ids = rq->tool_ids.data();
  rq->req.n_dirs = rq->n_dirs.data();
  rq->req.dirs = rq->dirs.data();
  if (r->n_fixture_sets > 0) {
    rq->fixture_of.assign(r->fixture_of, r->fixture_of + nd);
    rq->req.fixture_of = rq->fixture_of.data();
  }
  STCHK(imf_query_footprint(c, &rq->req, &rq->footprint));
  rq->t_submit = std::chrono::steady_clock::now();
  {
    std::lock_guard<std::mutex> lk(c->smu);
    if (c->queue.size() >= 4096) return fail(IMF_EBUSY, "serving queue full");
    if (c->workers.empty())
      for (int i = 0; i < c->max_inflight; i++) c->workers.emplace_back(serve_worker, c);
    rq->ticket = c->next_ticket++;
    c->reqs[rq->ticket] = rq;
    c->queue.push_back(rq);
    *ticket = rq->ticket;
  }
  c->scv.notify_all();
  return IMF_OK;
}

extern "C" imf_status imf_wait(imf_ctx* c, uint64_t ticket, int timeout_ms, imf_stats* st) {
  if (!c) return fail(IMF_EINVAL, "ctx is NULL");
  std::unique_lock<std::mutex> lk(c->smu);
  auto it = c->reqs.find(ticket);
  if (it == c->reqs.end()) return fail(IMF_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  auto rq = it->second;
  auto done = [&] { return rq->state >= 2; };
  if (timeout_ms < 0) {
    c->scv.wait(lk, done);
  } else if (!c->scv.wait_for(lk, std::chrono::milliseconds(timeout_ms), done)) {
    return fail(IMF_ETIMEOUT, "request %llu still running", (unsigned long long)ticket);
  }
  c->reqs.erase(ticket);
  if (st) *st = rq->stats;
  if (rq->state == 3) return fail(IMF_ECANCELLED, "request %llu was cancelled", (unsigned long long)ticket);
  if (rq->status != IMF_OK) {
    g_err = rq->err;
    return rq->status;
  }
  return IMF_OK;
}

extern "C" imf_status imf_cancel(imf_ctx* c, uint64_t ticket) {
  if (!c) return fail(IMF_EINVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(c->smu);
  auto it = c->reqs.find(ticket);
  if (it == c->reqs.end()) return fail(IMF_EINVAL, "unknown ticket");
  auto rq = it->second;
  if (rq->state != 0) return fail(IMF_EBUSY, "request already started");
  for (auto q = c->queue.begin(); q != c->queue.end(); ++q)
    if ((*q)->ticket == ticket) {
      c->queue.erase(q);
      break;
    }
  rq->state = 3;
  c->scv.notify_all();
  return IMF_OK;
}
