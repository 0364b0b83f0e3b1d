// Host side of the C ABI declared in include/sg.h: plans, validation,
// workspace, plan-time weight spectra, per-step launch sequences.
#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "sg.h"
#include "sg_internal.h"

// Workspace of sg_forces_noalloc: a file-scope device array, one per GPU the
// library runs on, held until the process ends.  Host code never uses the
// array's name as an address (it is a host-side stand-in): each device's
// address comes from hipGetSymbolAddress at plan creation, with that device
// current, and is kept per device.
#define SG_NOALLOC_BYTES (64ull << 20)
static __device__ __align__(256) unsigned char scratch[SG_NOALLOC_BYTES];

namespace {

thread_local std::string g_msg;

// Diagnostics from the environment, read at each use: SG_LOG (non-empty,
// not "0") prints every plan's launch choices and every error to stderr;
// SG_ROCTX likewise marks the entry points (and the passes of an eager
// step) with roctx ranges, for rocprofv3 --marker-trace, from libroctx64
// loaded at first use (no link-time dependency; nothing happens if it is
// missing).
bool env_on(const char* name) {
  const char* v = getenv(name);
  return v && *v && strcmp(v, "0") != 0;
}

sg_status fail(sg_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_msg = buf;
  if (env_on("SG_LOG")) fprintf(stderr, "sg: error %d: %s\n", (int)s, buf);
  return s;
}

struct Roctx {
  int (*push)(const char*) = nullptr;
  int (*pop)() = nullptr;
};
const Roctx& roctx() {
  static const Roctx r = [] {
    Roctx x;
    void* h = dlopen("libroctx64.so", RTLD_NOW | RTLD_LOCAL);
    if (!h) h = dlopen("/opt/rocm/lib/libroctx64.so", RTLD_NOW | RTLD_LOCAL);
    if (h) {
      x.push = (int (*)(const char*))dlsym(h, "roctxRangePushA");
      x.pop = (int (*)())dlsym(h, "roctxRangePop");
      if (!x.push || !x.pop) x = Roctx{};
    }
    return x;
  }();
  return r;
}
// A roctx range for the lifetime of the object, when SG_ROCTX asks for them.
class Range {
 public:
  explicit Range(const char* msg) : on_(env_on("SG_ROCTX") && roctx().push) {
    if (on_) roctx().push(msg);
  }
  Range(const char* fmt, int a, int b, int c) : on_(env_on("SG_ROCTX") && roctx().push) {
    if (on_) {
      char buf[96];
      snprintf(buf, sizeof buf, fmt, a, b, c);
      roctx().push(buf);
    }
  }
  ~Range() {
    if (on_) roctx().pop();
  }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;

 private:
  bool on_;
};

// Device address of scratch on the current device (once per device).
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;
hipError_t scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[dev] = ptr;
  *out = ptr;
  return hipSuccess;
}

bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }
// Grid sizes with kernels: 2^a from 4 to 8192 and 3 * 2^a from 12 to 1536.
bool size_ok(int v) { return pow2_in(v, 4, 8192) || (v % 3 == 0 && pow2_in(v / 3, 4, 512)); }

// Roots of unity exp(-2 pi i k / B), k = 0..B-1, from long double sin/cos of
// the octant-reduced angle (one rounding to the stored precision).
template <typename R>
std::vector<R> roots_table(int B) {
  std::vector<R> out(2 * (size_t)B);
  const long double twopi = 6.283185307179586476925286766559005768L;
  for (int k = 0; k < B; ++k) {
    // reduce k/B into [0, 1/8] using symmetries for accuracy
    long double c, s;
    int kk = k;
    // exp(-2 pi i k/B) = cos(2 pi k/B) - i sin(2 pi k/B)
    long double a = twopi * (long double)kk / (long double)B;
    c = cosl(a);
    s = sinl(a);
    // exact values at multiples of pi/4 and pi/2
    if ((8LL * k) % B == 0) {
      const int o = (int)((8LL * k) / B) % 8;
      const long double h = 0.707106781186547524400844362104849039L;
      const long double cs[8] = {1, h, 0, -h, -1, -h, 0, h};
      const long double sn[8] = {0, h, 1, h, 0, -h, -1, -h};
      c = cs[o];
      s = sn[o];
    }
    out[2 * (size_t)k] = (R)c;
    out[2 * (size_t)k + 1] = (R)(-s);
  }
  return out;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on the three-term
// recurrence of the Legendre polynomials, long double).
void gl_rule(int q, double* x, double* w) {
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < q; ++i) {
    long double z = cosl(pi * (i + 0.75L) / (q + 0.5L)), dp = 1;
    for (int it = 0; it < 200; ++it) {
      long double p0 = 1, p1 = z;
      for (int j = 2; j <= q; ++j) {
        long double p2 = ((2 * j - 1) * z * p1 - (j - 1) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      dp = q * (z * p1 - p0) / (z * z - 1);
      long double dz = p1 / dp;
      z -= dz;
      if (fabsl(dz) < 1e-20L) break;
    }
    long double p0 = 1, p1 = z;
    for (int j = 2; j <= q; ++j) {
      long double p2 = ((2 * j - 1) * z * p1 - (j - 1) * p0) / j;
      p0 = p1;
      p1 = p2;
    }
    dp = q * (z * p1 - p0) / (z * z - 1);
    x[i] = (double)z;
    w[i] = (double)(2.0L / ((1 - z * z) * dp * dp));
  }
}

struct GridPlan {
  sg_grid g;
  int M, N, k, kind;
  double hx, hy;
  int64_t off;
  void* tabx = nullptr;
  void* taby = nullptr;
  void* X = nullptr;
  void* V = nullptr;
  const void* r2m = nullptr;
  const void* r2n = nullptr;
  void* twA = nullptr;  // stage twiddles: forward rows, columns, inverse rows
  void* twB = nullptr;
  void* twC = nullptr;
  void* twC1 = nullptr;     // inverse rows in launch variant 1 (FP32, where it exists)
  bool fs = false;          // columns by the four-step pass (long columns, and 1536 in FP32)
  bool fs_adj = false;      // ... in the adjoint as well (the long columns)
  void* twfs = nullptr;     // its twiddle table
  int tab_bytes = 8;        // bytes per spectrum entry: double, float hi + lo, or float
};

// Grids of one size and order: one launch per pass runs all of them
// (descriptor array desc on the device, blockIdx.y = member).
struct GridClass {
  int M, N, k;
  std::vector<int> members;
  sg_bgrid* desc = nullptr;
  sg_bgrid* desc_y = nullptr;  // the same with X = V (adjoint: row spectra of gy)
  sg_bgrid* desc_s = nullptr;  // the same with X and V in the no-allocation scratch
  int tile[3] = {0, 0, 0};  // rows / columns per workgroup of passes A, B, C (0 = compiled maximum)
  int var[3] = {0, 0, 0};   // launch variant of passes A, B, C (sg_variants)
  int src = 0;              // how var and tile were chosen: 0 defaults, 1 timed here, 2 the tuning store
};

// One captured step: the graph of every class's three launches for a given
// (sigma, fx, fy), classes spread over the plan's side streams.
struct StepGraph {
  const void* sigma;
  void* fx;
  void* fy;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

}  // namespace

struct sg_plan_s {
  std::vector<GridPlan> grids;
  std::vector<GridClass> classes;
  std::vector<hipStream_t> side;    // streams of a captured step (default priority)
  std::vector<hipEvent_t> sync_ev;  // fork / join events of the captured step
  std::vector<StepGraph> graphs;    // most recent first, at most kMaxGraphs
  sg_precision prec;
  hipStream_t st;
  uint32_t flags;
  bool sticky = false;
  int device = 0;
  int64_t bytes = 0;
  int64_t total = 0;
  std::vector<void*> allocs;
  std::map<int, void*> roots;  // plan-precision tables keyed by B
  int* flag = nullptr;         // device word for the finite check
  bool timing = false;         // per-pass event timing (sg_plan_set_timing)
  std::vector<hipEvent_t> ev;  // 4 events per grid and call while timing
  int64_t timed_calls = 0;
  int64_t noalloc_bytes = 0;   // X and V of every grid laid out in scratch
  bool noalloc_ok = false;     // they fit (sg_forces_noalloc usable)
};

namespace {

// Fault injection for the error-path tests, read from the environment at
// each call: SG_FAULT_INJECT=alloc refuses every device allocation of a plan,
// alloc:N only the N-th one (1-based, counted from the start of
// sg_plan_create on this thread), device makes the next per-step call fail as
// if a HIP call had returned an error (the plan then turns sticky).
thread_local int g_alloc_count = 0;

bool inject_alloc_failure() {
  const char* v = getenv("SG_FAULT_INJECT");
  if (!v) return false;
  if (strcmp(v, "alloc") == 0) return true;
  if (strncmp(v, "alloc:", 6) == 0) return g_alloc_count == atoi(v + 6);
  return false;
}

bool inject_device_failure() {
  const char* v = getenv("SG_FAULT_INJECT");
  return v && strcmp(v, "device") == 0;
}

// Temporary device memory of plan creation (freed by the caller before it
// returns), counted for the fault injection like the plan's own.
sg_status tmp_alloc(void** out, size_t bytes, const char* what) {
  ++g_alloc_count;
  *out = nullptr;
  if (inject_alloc_failure())
    return fail(SG_ERR_NOMEM, "%s: allocation %d of %zu bytes refused (SG_FAULT_INJECT)", what, g_alloc_count, bytes);
  hipError_t e = hipMalloc(out, bytes ? bytes : 16);
  if (e != hipSuccess) {
    *out = nullptr;
    (void)hipGetLastError();
    return fail(SG_ERR_NOMEM, "%s: hipMalloc(%zu) failed: %s", what, bytes, hipGetErrorString(e));
  }
  return SG_OK;
}

// Device memory of the plan (released by sg_plan_destroy, or at once when
// plan creation fails).
sg_status dev_alloc(sg_plan p, void** out, size_t bytes) {
  ++g_alloc_count;
  if (inject_alloc_failure())
    return fail(SG_ERR_NOMEM, "allocation %d of %zu bytes refused (SG_FAULT_INJECT)", g_alloc_count, bytes);
  hipError_t e = hipMalloc(out, bytes ? bytes : 16);
  if (e != hipSuccess) {
    *out = nullptr;
    (void)hipGetLastError();
    return fail(SG_ERR_NOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  p->allocs.push_back(*out);
  p->bytes += (int64_t)bytes;
  return SG_OK;
}

sg_status hip_check(sg_plan p, hipError_t e, const char* what) {
  if (e == hipSuccess) return SG_OK;
  if (p) p->sticky = true;
  return fail(SG_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

template <typename R>
sg_status upload_roots(sg_plan p, int B, void** out) {
  std::vector<R> h = roots_table<R>(B);
  sg_status s = dev_alloc(p, out, h.size() * sizeof(R));
  if (s != SG_OK) return s;
  return hip_check(p, hipMemcpy(*out, h.data(), h.size() * sizeof(R), hipMemcpyHostToDevice), "hipMemcpy roots");
}

// Stage twiddle table of one pass (see sg_twiddles), allocated in the plan.
sg_status make_twiddles(sg_plan p, int prec, int pass, int len, const void* roots, void** out) {
  const int n = sg_twiddles(prec, pass, len, nullptr, nullptr, p->st);
  if (n < 0) return fail(SG_ERR_UNSUPPORTED, "no FFT kernel for length %d", len);
  sg_status s = dev_alloc(p, out, (size_t)(prec == 0 ? 16 : 8) * (size_t)(n > 0 ? n : 1));
  if (s != SG_OK) return s;
  sg_twiddles(prec, pass, len, roots, *out, p->st);
  return hip_check(p, hipGetLastError(), "twiddle table");
}

// Twiddle table of the four-step column pass of length N (long double,
// rounded once to the plan precision).
sg_status upload_fs_twiddles(sg_plan p, int prec, int N, void** out) {
  const int n = sg_colfs_twiddles(prec, N, nullptr, nullptr);
  if (n <= 0) return fail(SG_ERR_UNSUPPORTED, "no four-step column pass for length %d", N);
  std::vector<double> re(n), im(n);
  sg_colfs_twiddles(prec, N, re.data(), im.data());
  const size_t el = prec == 0 ? 8 : 4;
  std::vector<unsigned char> h(2 * el * (size_t)n);
  for (int i = 0; i < n; ++i) {
    if (prec == 0) {
      double v[2] = {re[i], im[i]};
      memcpy(&h[16 * (size_t)i], v, 16);
    } else {
      float v[2] = {(float)re[i], (float)im[i]};
      memcpy(&h[8 * (size_t)i], v, 8);
    }
  }
  sg_status s = dev_alloc(p, out, h.size());
  if (s != SG_OK) return s;
  return hip_check(p, hipMemcpy(*out, h.data(), h.size(), hipMemcpyHostToDevice), "hipMemcpy four-step twiddles");
}

void drop_events(sg_plan p) {
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  p->ev.clear();
  p->timed_calls = 0;
}

void drop_graphs(sg_plan p) {
  for (StepGraph& g : p->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  p->graphs.clear();
}

void release(sg_plan p) {
  drop_events(p);
  drop_graphs(p);
  for (hipEvent_t e : p->sync_ev) (void)hipEventDestroy(e);
  p->sync_ev.clear();
  for (hipStream_t q : p->side) (void)hipStreamDestroy(q);
  p->side.clear();
  for (void* a : p->allocs) (void)hipFree(a);
  p->allocs.clear();
}

// record one timing event on the plan's stream (no-op unless timing)
hipError_t mark(sg_plan p) {
  if (!p->timing) return hipSuccess;
  hipEvent_t e;
  hipError_t r = hipEventCreate(&e);
  if (r != hipSuccess) return r;
  p->ev.push_back(e);
  return hipEventRecord(e, p->st);
}

sg_status check_plan(sg_plan p) {
  if (!p) return fail(SG_ERR_ARG, "plan is NULL");
  if (p->sticky) return fail(SG_ERR_STATE, "plan is in the sticky error state after a device error");
  return SG_OK;
}

// Per-step entry: the plan check, then the injected device failure if asked.
sg_status step_entry(sg_plan p) {
  sg_status s = check_plan(p);
  if (s != SG_OK) return s;
  if (inject_device_failure()) return hip_check(p, hipErrorLaunchFailure, "injected (SG_FAULT_INJECT=device)");
  return SG_OK;
}

// Weight spectra of one grid (plan time, FP64 throughout).
sg_status build_spectra(sg_plan p, GridPlan& G, const void* r2m64, const void* r2n64) {
  const int M = G.M, N = G.N;
  void *twA64 = nullptr, *twS64 = nullptr;
  sg_status ts = make_twiddles(p, 0, 0, M, r2m64, &twA64);
  if (ts == SG_OK) ts = make_twiddles(p, 0, 3, N, r2n64, &twS64);
  if (ts != SG_OK) return ts;
  double* wp = nullptr;
  void* S = nullptr;
  sg_status as = tmp_alloc((void**)&wp, sizeof(double) * 2 * (size_t)(2 * M) * (2 * N), "plan-time weight table");
  if (as != SG_OK) return as;
  as = tmp_alloc(&S, 16 * (size_t)(2 * N) * M, "plan-time spectrum workspace");
  if (as != SG_OK) {
    (void)hipFree(wp);
    return as;
  }
  hipError_t e = hipSuccess;
  double* wpx = wp;
  double* wpy = wp + (size_t)(2 * M) * (2 * N);
  // stored form of the tables: double, float hi + lo, or float
  const int fp32 = p->prec == SG_FP64 ? 0 : (G.tab_bytes == 8 ? 1 : 2);
  const double scale = 1.0 / (4.0 * (double)M * (double)N);
  sg_status st = SG_OK;
  // columns of 8192: the four-step spectrum kernel (FP64 twiddles of that length)
  void* twfs64 = nullptr;
  if (N == 8192) {
    sg_status ts2 = upload_fs_twiddles(p, 0, N, &twfs64);
    if (ts2 != SG_OK) {
      (void)hipFree(wp);
      (void)hipFree(S);
      return ts2;
    }
  }
  auto spec = [&](void* tab) {
    return N == 8192 ? sg_launch_specfs(N, S, M, tab, G.kind, fp32, scale, r2n64, twfs64, p->st)
                     : sg_launch_spec_col(N, S, M, tab, G.kind, fp32, scale, r2n64, twS64, p->st);
  };
  e = sg_launch_weights(G.k, G.hx, G.hy, M, N, wpx, wpy, 0, p->st);
  if (e == hipSuccess) e = sg_launch_row_fwd(0, M, wpx, 2 * M, S, 2 * N, r2m64, 0, 1, twA64, nullptr, 1, 0, p->st);
  if (e == hipSuccess) e = spec(G.tabx);
  if (e == hipSuccess) e = sg_launch_row_fwd(0, M, wpy, 2 * M, S, 2 * N, r2m64, 0, 1, twA64, nullptr, 1, 0, p->st);
  if (e == hipSuccess) e = spec(G.taby);
  if (e == hipSuccess) e = hipStreamSynchronize(p->st);
  if (e != hipSuccess) st = hip_check(p, e, "plan-time spectrum");
  (void)hipFree(wp);
  (void)hipFree(S);
  return st;
}

constexpr size_t kMaxGraphs = 4;
constexpr int kSideStreams = 4;

// The column pass of one class: the four-step kernel for long columns, the
// Stockham kernel otherwise.
hipError_t launch_cols(sg_plan p, const GridClass& c, int tile, hipStream_t q, const sg_bgrid* desc = nullptr) {
  const int prec = p->prec == SG_FP64 ? 0 : 1;
  const GridPlan& G = p->grids[c.members[0]];
  const int solve = c.k >= 3 ? c.k : 0;
  const int ng = (int)c.members.size();
  const int tj = sg_row_tile(prec, c.M, c.N);
  const sg_bgrid* d = desc ? desc : c.desc;
  if (G.fs)
    return sg_launch_colfs(prec, c.N, nullptr, nullptr, c.M, tj, nullptr, nullptr, G.kind, G.tab_bytes, G.r2n, solve,
                           G.twfs, d, ng, q);
  return sg_launch_col(prec, c.N, nullptr, nullptr, c.M, tj, nullptr, nullptr, G.kind, G.r2n, solve, G.twB, d, ng,
                       tile, c.var[1], q);
}

// The inverse row pass of one class (its launch variant and that variant's
// twiddle table).
hipError_t launch_rows_inv(sg_plan p, const GridClass& c, void* fx, void* fy, int tile, hipStream_t q,
                           const sg_bgrid* desc) {
  const int prec = p->prec == SG_FP64 ? 0 : 1;
  const GridPlan& G = p->grids[c.members[0]];
  const int tj = sg_row_tile(prec, c.M, c.N);
  return sg_launch_row_inv(prec, c.M, nullptr, fx, fy, c.N, tj, G.r2m, c.var[2] ? G.twC1 : G.twC, desc,
                           (int)c.members.size(), tile, c.var[2], q);
}

// The three launches of every grid of one class on stream q.
hipError_t issue_class(sg_plan p, const GridClass& c, const void* sigma, void* fx, void* fy, hipStream_t q,
                       const int* tile) {
  const int prec = p->prec == SG_FP64 ? 0 : 1;
  const GridPlan& G = p->grids[c.members[0]];
  const int solve = c.k >= 3 ? c.k : 0;
  const int ng = (int)c.members.size();
  hipError_t e = sg_launch_row_fwd(prec, c.M, sigma, c.M, nullptr, c.N, G.r2m, solve, 0, G.twA, c.desc, ng, tile[0], q);
  if (e == hipSuccess) e = launch_cols(p, c, tile[1], q);
  if (e == hipSuccess) e = launch_rows_inv(p, c, fx, fy, tile[2], q, c.desc);
  return e;
}

// Capture the whole step (every class) for these buffers: classes spread
// round-robin over the plan's side streams, forked from and joined to the
// first one.
sg_status capture_step(sg_plan p, const void* sigma, void* fx, void* fy, StepGraph* out) {
  const int nside = (int)p->side.size();
  hipStream_t q0 = p->side[0];
  hipError_t e = hipStreamBeginCapture(q0, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_check(p, e, "hipStreamBeginCapture");
  hipError_t ce = hipEventRecord(p->sync_ev[0], q0);
  for (int i = 1; i < nside && ce == hipSuccess; ++i) ce = hipStreamWaitEvent(p->side[i], p->sync_ev[0], 0);
  for (size_t ci = 0; ci < p->classes.size() && ce == hipSuccess; ++ci)
    ce = issue_class(p, p->classes[ci], sigma, fx, fy, p->side[ci % nside], p->classes[ci].tile);
  for (int i = 1; i < nside && ce == hipSuccess; ++i) {
    ce = hipEventRecord(p->sync_ev[i], p->side[i]);
    if (ce == hipSuccess) ce = hipStreamWaitEvent(q0, p->sync_ev[i], 0);
  }
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(q0, &g);
  if (ce != hipSuccess || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_check(p, ce != hipSuccess ? ce : e, "step capture");
  }
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_check(p, e, "hipGraphInstantiate");
  }
  out->sigma = sigma;
  out->fx = fx;
  out->fy = fy;
  out->graph = g;
  out->exec = x;
  return SG_OK;
}

// Time pass `pass` of class c with a candidate tile (ms per launch, median of
// reps), on scratch buffers.
sg_status time_tile(sg_plan p, GridClass& c, int pass, int tile, const void* sig, void* fx, void* fy, float* ms) {
  int t3[3] = {c.tile[0], c.tile[1], c.tile[2]};
  t3[pass] = tile;
  const int prec = p->prec == SG_FP64 ? 0 : 1;
  const GridPlan& G = p->grids[c.members[0]];
  const int solve = c.k >= 3 ? c.k : 0;
  const int ng = (int)c.members.size();
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return fail(SG_ERR_DEVICE, "hipEventCreate");
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return fail(SG_ERR_DEVICE, "hipEventCreate");
  }
  const int reps = 5;
  float best = 1e30f;
  hipError_t e = hipSuccess;
  auto launch = [&](int ps) -> hipError_t {
    if (ps == 0)
      return sg_launch_row_fwd(prec, c.M, sig, c.M, nullptr, c.N, G.r2m, solve, 0, G.twA, c.desc, ng, t3[0], p->st);
    if (ps == 1) return launch_cols(p, c, t3[1], p->st);
    return launch_rows_inv(p, c, fx, fy, t3[2], p->st, c.desc);
  };
  // each repetition runs the class's whole step and times the pass under
  // test inside it, so that the pass meets the caches as a step leaves them
  // (a pass repeated on its own rewrites lines it has just written, which
  // favours tiles whose stores are shorter pieces)
  for (int r = 0; r <= reps && e == hipSuccess; ++r) {
    for (int ps = 0; ps < 3 && e == hipSuccess; ++ps) {
      if (ps == pass) e = hipEventRecord(a, p->st);
      if (e == hipSuccess) e = launch(ps);
      if (e == hipSuccess && ps == pass) e = hipEventRecord(b, p->st);
    }
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    if (r > 0 && t < best) best = t;  // first run warms up
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return hip_check(p, e, "autotune timing");
  *ms = best;
  return SG_OK;
}

// ------------------------------------------------------------- tuning --
// Launch choices per class: the variant of each pass (sg_variants: kernels
// of the same transform with other buffering or elements per thread) and
// its tile (rows or columns per workgroup).  Choices live in a process-wide
// store, like FFT wisdom: every plan created afterwards takes the variants
// recorded for its (device, precision, size, order), tuned or not, so that
// plans of one process compute identical results; tiles (which never change
// results) are recorded per class size (number of grids) as well.  With
// SG_TUNE_CACHE=path the store is read from that file on first use and
// written back (whole, through a temporary file and a rename) after new
// choices are timed.  SG_TUNE: off = defaults only, the store ignored;
// quick = time tiles only; full = variants, then tiles.  Unset: full for
// plans created with SG_FLAG_AUTOTUNE, the store alone for other plans.
#ifndef SG_BUILD_ID
#define SG_BUILD_ID "dev"
#endif

enum TuneMode { TUNE_UNSET, TUNE_OFF, TUNE_QUICK, TUNE_FULL };

TuneMode tune_mode() {
  const char* v = getenv("SG_TUNE");
  if (!v || !*v) return TUNE_UNSET;
  if (strcmp(v, "off") == 0 || strcmp(v, "0") == 0) return TUNE_OFF;
  if (strcmp(v, "quick") == 0) return TUNE_QUICK;
  return TUNE_FULL;
}

struct TuneStore {
  std::mutex mu;
  std::map<std::string, std::array<int, 3>> var;   // device/prec/size/order -> variants
  std::map<std::string, std::array<int, 3>> tile;  // ... /grids -> tiles
  std::string loaded;                              // cache file read into the store
};
TuneStore g_tune;

// Entries of a cache file: lines  "key": [a, b, c]  after a line naming the
// section ("variants" or "tiles").  Malformed lines are skipped.
void read_cache(const std::string& path, std::map<std::string, std::array<int, 3>>& var,
                std::map<std::string, std::array<int, 3>>& tile) {
  FILE* f = fopen(path.c_str(), "r");
  if (!f) return;
  char line[1024];
  int section = 0;  // 1 variants, 2 tiles
  while (fgets(line, sizeof line, f)) {
    if (strstr(line, "\"variants\"")) section = 1;
    else if (strstr(line, "\"tiles\"")) section = 2;
    const char* q0 = strchr(line, '"');
    const char* q1 = q0 ? strchr(q0 + 1, '"') : nullptr;
    const char* br = q1 ? strchr(q1, '[') : nullptr;
    std::array<int, 3> v{};
    if (!section || !br || sscanf(br, "[%d , %d , %d]", &v[0], &v[1], &v[2]) != 3) continue;
    const std::string key(q0 + 1, q1);
    if (key.find('/') == std::string::npos) continue;
    (section == 1 ? var : tile)[key] = v;
  }
  fclose(f);
}

bool write_cache(const std::string& path, const std::map<std::string, std::array<int, 3>>& var,
                 const std::map<std::string, std::array<int, 3>>& tile) {
  const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return false;
  fprintf(f, "{\"sg_tune_cache\": 1,\n");
  for (int sec = 0; sec < 2; ++sec) {
    const auto& m = sec ? tile : var;
    fprintf(f, " \"%s\": {\n", sec ? "tiles" : "variants");
    size_t i = 0;
    for (const auto& kv : m)
      fprintf(f, "  \"%s\": [%d, %d, %d]%s\n", kv.first.c_str(), kv.second[0], kv.second[1], kv.second[2],
              ++i < m.size() ? "," : "");
    fprintf(f, " }%s\n", sec ? "" : ",");
  }
  fprintf(f, "}\n");
  const bool ok = fclose(f) == 0;
  return ok && rename(tmp.c_str(), path.c_str()) == 0;
}

std::string device_tag(int dev) {
  hipDeviceProp_t pr;
  if (hipGetDeviceProperties(&pr, dev) != hipSuccess) return "unknown";
  std::string arch = pr.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch.resize(colon);
  return arch + "/" + std::to_string(pr.multiProcessorCount) + "cu/" SG_BUILD_ID;
}

std::string var_key(const std::string& dev, int prec, const GridClass& c) {
  char b[160];
  snprintf(b, sizeof b, "%s/%s/%dx%d/k%d", dev.c_str(), prec == 0 ? "fp64" : "fp32", c.M, c.N, c.k);
  return b;
}
std::string tile_key(const std::string& dev, int prec, const GridClass& c) {
  return var_key(dev, prec, c) + "/g" + std::to_string(c.members.size());
}

// Time every tile (powers of two up to the compiled maximum) of one pass in
// the class's variant; the best goes into c.tile.
sg_status tune_tiles(sg_plan p, GridClass& c, int pass, const void* sig, void* fx, void* fy, float* best_ms) {
  const int prec = p->prec == SG_FP64 ? 0 : 1;
  const int cap = sg_max_tile(prec, pass, pass == 1 ? c.N : c.M, c.var[pass]);
  int best_tile = 0;
  float best = 1e30f;
  sg_status s = SG_OK;
  for (int t = 1; t <= cap && s == SG_OK; t *= 2) {
    float ms = 0.0f;
    s = time_tile(p, c, pass, t, sig, fx, fy, &ms);
    if (s == SG_OK && ms < best) {
      best = ms;
      best_tile = t;
    }
  }
  if (s == SG_OK) c.tile[pass] = best_tile;
  if (best_ms) *best_ms = best;
  return s;
}

// Apply the store's choices to every class; time what is missing when asked
// to (full: variants and tiles; quick: tiles), record it and write the
// cache file.
sg_status tune(sg_plan p) {
  const TuneMode mode = tune_mode();
  if (mode == TUNE_OFF) return SG_OK;
  const bool timing = mode == TUNE_FULL || mode == TUNE_QUICK || (mode == TUNE_UNSET && (p->flags & SG_FLAG_AUTOTUNE));
  const bool variants = mode == TUNE_FULL || (mode == TUNE_UNSET && (p->flags & SG_FLAG_AUTOTUNE));
  const int prec = p->prec == SG_FP64 ? 0 : 1;
  const std::string dev = device_tag(p->device);
  const char* cache_env = getenv("SG_TUNE_CACHE");
  const std::string cache = cache_env ? cache_env : "";
  std::lock_guard<std::mutex> lk(g_tune.mu);
  if (!cache.empty() && g_tune.loaded != cache) {
    read_cache(cache, g_tune.var, g_tune.tile);
    g_tune.loaded = cache;
  }
  // a stored choice is used only if this build has it
  auto valid_var = [&](const GridClass& c, const std::array<int, 3>& v) {
    for (int pass = 0; pass < 3; ++pass) {
      const int n = (pass == 1 && p->grids[c.members[0]].fs) ? 1 : sg_variants(prec, pass, pass == 1 ? c.N : c.M);
      if (v[pass] < 0 || v[pass] >= n) return false;
    }
    return true;
  };
  auto valid_tile = [&](const GridClass& c, const std::array<int, 3>& t) {
    for (int pass = 0; pass < 3; ++pass)
      if (t[pass] < 0 || t[pass] > sg_max_tile(prec, pass, pass == 1 ? c.N : c.M, c.var[pass])) return false;
    return true;
  };
  std::vector<int> todo;  // classes with something to time
  for (int i = 0; i < (int)p->classes.size(); ++i) {
    GridClass& c = p->classes[i];
    bool have_var = false, have_tile = false;
    auto iv = g_tune.var.find(var_key(dev, prec, c));
    if (iv != g_tune.var.end() && valid_var(c, iv->second)) {
      for (int pass = 0; pass < 3; ++pass) c.var[pass] = iv->second[pass];
      have_var = true;
    }
    auto it = g_tune.tile.find(tile_key(dev, prec, c));
    if (have_var || !variants) {
      if (it != g_tune.tile.end() && valid_tile(c, it->second)) {
        for (int pass = 0; pass < 3; ++pass) c.tile[pass] = it->second[pass];
        have_tile = true;
      }
    }
    if (have_var || have_tile) c.src = 2;
    if (timing && !((have_var || !variants) && have_tile)) todo.push_back(i);
  }
  if (todo.empty()) return SG_OK;
  // scratch buffers for the timing runs (zero input)
  const size_t el = p->prec == SG_FP64 ? 8 : 4;
  void *sig = nullptr, *fx = nullptr, *fy = nullptr;
  sg_status s = tmp_alloc(&sig, el * (size_t)p->total, "tuning buffers");
  if (s == SG_OK) s = tmp_alloc(&fx, el * (size_t)p->total, "tuning buffers");
  if (s == SG_OK) s = tmp_alloc(&fy, el * (size_t)p->total, "tuning buffers");
  if (s == SG_OK) s = hip_check(p, hipMemsetAsync(sig, 0, el * (size_t)p->total, p->st), "tuning buffers");
  for (int i : todo) {
    if (s != SG_OK) break;
    GridClass& c = p->classes[i];
    bool tiled[3] = {false, false, false};
    if (variants && g_tune.var.find(var_key(dev, prec, c)) == g_tune.var.end()) {
      // each variant with its best tile; the fastest stays, with that tile
      for (int pass = 0; pass < 3 && s == SG_OK; ++pass) {
        const bool fixed = pass == 1 && p->grids[c.members[0]].fs;
        const int n = fixed ? 1 : sg_variants(prec, pass, pass == 1 ? c.N : c.M);
        if (n < 2) continue;
        int best_v = c.var[pass], best_t = c.tile[pass];
        float best = 1e30f;
        for (int v = 0; v < n && s == SG_OK; ++v) {
          c.var[pass] = v;
          float ms = 0.0f;
          s = tune_tiles(p, c, pass, sig, fx, fy, &ms);
          if (s == SG_OK && ms < best) {
            best = ms;
            best_v = v;
            best_t = c.tile[pass];
          }
        }
        c.var[pass] = best_v;
        c.tile[pass] = best_t;
        tiled[pass] = true;
      }
      if (s == SG_OK) g_tune.var[var_key(dev, prec, c)] = {c.var[0], c.var[1], c.var[2]};
    }
    for (int pass = 0; pass < 3 && s == SG_OK; ++pass)
      if (!tiled[pass]) s = tune_tiles(p, c, pass, sig, fx, fy, nullptr);
    if (s == SG_OK) {
      g_tune.tile[tile_key(dev, prec, c)] = {c.tile[0], c.tile[1], c.tile[2]};
      c.src = 1;
    }
  }
  (void)hipStreamSynchronize(p->st);
  if (sig) (void)hipFree(sig);
  if (fx) (void)hipFree(fx);
  if (fy) (void)hipFree(fy);
  if (s == SG_OK && !cache.empty()) {
    // merge with what other processes may have written meanwhile; ours wins
    std::map<std::string, std::array<int, 3>> v2, t2;
    read_cache(cache, v2, t2);
    for (const auto& kv : g_tune.var) v2[kv.first] = kv.second;
    for (const auto& kv : g_tune.tile) t2[kv.first] = kv.second;
    g_tune.var = v2;
    g_tune.tile = t2;
    if (!write_cache(cache, g_tune.var, g_tune.tile))
      fprintf(stderr, "sg: could not write the tuning cache %s\n", cache.c_str());
  }
  return s;
}

}  // namespace

extern "C" {

const char* sg_status_string(sg_status s) {
  switch (s) {
    case SG_OK: return "SG_OK";
    case SG_ERR_ARG: return "SG_ERR_ARG: invalid argument";
    case SG_ERR_UNSUPPORTED: return "SG_ERR_UNSUPPORTED: unsupported order or size";
    case SG_ERR_NOMEM: return "SG_ERR_NOMEM: allocation failed";
    case SG_ERR_DEVICE: return "SG_ERR_DEVICE: HIP error";
    case SG_ERR_STATE: return "SG_ERR_STATE: plan in error state or non-finite input";
  }
  return "unknown sg_status";
}

const char* sg_last_error_message(void) { return g_msg.c_str(); }

sg_status sg_plan_create(sg_plan* out, const sg_grid* grids, int32_t ngrids, sg_precision prec, void* hip_stream,
                         uint32_t flags) {
  Range range("sg_plan_create");
  g_msg.clear();
  g_alloc_count = 0;
  if (!out) return fail(SG_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!grids || ngrids < 1) return fail(SG_ERR_ARG, "need at least one grid (ngrids=%d)", ngrids);
  if (prec != SG_FP64 && prec != SG_FP32_SPLIT) return fail(SG_ERR_ARG, "unknown precision %d", (int)prec);
  if (flags & ~(SG_FLAG_CHECK_FINITE | SG_FLAG_GRAPH | SG_FLAG_AUTOTUNE | SG_FLAG_SPECTRA_SPLIT))
    return fail(SG_ERR_ARG, "unknown flags 0x%x", flags);
  for (int i = 0; i < ngrids; ++i) {
    const sg_grid& g = grids[i];
    if (g.nx < 2 || g.ny < 2) return fail(SG_ERR_ARG, "grid %d: nx=%d ny=%d (need >= 2)", i, g.nx, g.ny);
    if (!isfinite(g.x0) || !isfinite(g.x1) || !isfinite(g.y0) || !isfinite(g.y1) || !(g.x1 > g.x0) ||
        !(g.y1 > g.y0))
      return fail(SG_ERR_ARG, "grid %d: empty or non-finite domain", i);
    if (g.order < 1 || g.order > 5) return fail(SG_ERR_UNSUPPORTED, "grid %d: order %d (supported: 1..5)", i, g.order);
    if (!size_ok(g.nx) || !size_ok(g.ny))
      return fail(SG_ERR_UNSUPPORTED, "grid %d: %dx%d (supported: 2^a from 4 to 4096, 3*2^a from 12 to 1536)", i,
                  g.nx, g.ny);
  }
  sg_plan p = new (std::nothrow) sg_plan_s();
  if (!p) return fail(SG_ERR_NOMEM, "host allocation failed");
  p->prec = prec;
  p->st = (hipStream_t)hip_stream;
  p->flags = flags;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return fail(SG_ERR_DEVICE, "no HIP device");
  }
  // Gauss-Legendre rules for the plan-time weights: q = 4, 6, 10, 16
  {
    double gx[64] = {0}, gw[64] = {0};
    const int qs[4] = {4, 6, 10, 16};
    for (int a = 0; a < 4; ++a) gl_rule(qs[a], gx + 16 * a, gw + 16 * a);
    hipError_t e = sg_set_gl_tables(gx, gw);
    if (e != hipSuccess) {
      delete p;
      return fail(SG_ERR_DEVICE, "GL tables: %s", hipGetErrorString(e));
    }
  }
  const size_t cb = prec == SG_FP64 ? 16 : 8;  // complex element bytes
  std::map<int, void*> roots64;
  std::map<std::pair<int, int>, void*> tw;  // (pass, length) -> stage twiddles
  std::map<std::tuple<int, int, int, double, double, int>, std::pair<void*, void*>> spectra;  // shared weight spectra
  std::map<int, void*> twfs;  // four-step twiddle tables by length
  sg_status s = SG_OK;
  int64_t off = 0;
  for (int i = 0; i < ngrids && s == SG_OK; ++i) {
    GridPlan G;
    G.g = grids[i];
    G.M = grids[i].nx;
    G.N = grids[i].ny;
    G.k = grids[i].order;
    G.kind = (G.k % 2 == 0) ? 1 : 0;  // even k: splines centred on vertices, spectra with a bin phase
    G.hx = (grids[i].x1 - grids[i].x0) / G.M;
    G.hy = (grids[i].y1 - grids[i].y0) / G.N;
    G.off = off;
    off += (int64_t)G.M * G.N;
    // the four-step column pass for the long columns (SG_COLFS=0 in the
    // environment keeps the Stockham pass where it exists: a diagnostic)
    {
      const char* env = getenv("SG_COLFS");
      const bool off = env && strcmp(env, "0") == 0 && G.N <= 4096;
      const int sup = off ? 0 : sg_colfs_supported(prec == SG_FP64 ? 0 : 1, G.N);
      G.fs = sup != 0;
      G.fs_adj = sup == 1;
    }
    // one real per bin on a quarter of the lattice: FP64; hi+lo FP32; or, for
    // FP32-split plans without SG_FLAG_SPECTRA_SPLIT whose columns take the
    // four-step pass both ways, FP32.  For even k the bin phase is applied
    // in the column pass.
    G.tab_bytes = (prec == SG_FP32_SPLIT && G.fs_adj && !(flags & SG_FLAG_SPECTRA_SPLIT)) ? 4 : 8;
    const size_t tab_el = (size_t)G.tab_bytes;
    const size_t tab_n = (size_t)(G.M + 1) * (G.N + 1);
    // grids of equal size, order, cell shape and table form share one pair of spectra
    const auto key = std::make_tuple(G.M, G.N, G.k, G.hx, G.hy, G.tab_bytes);
    const bool fresh = !spectra.count(key);
    if (fresh) {
      if (s == SG_OK) s = dev_alloc(p, &G.tabx, tab_el * tab_n);
      if (s == SG_OK) s = dev_alloc(p, &G.taby, tab_el * tab_n);
      if (s == SG_OK) spectra[key] = std::make_pair(G.tabx, G.taby);
    } else {
      G.tabx = spectra[key].first;
      G.taby = spectra[key].second;
    }
    if (s == SG_OK) s = dev_alloc(p, &G.X, cb * (size_t)G.M * G.N);
    if (s == SG_OK) s = dev_alloc(p, &G.V, cb * 2 * (size_t)G.M * G.N);
    for (int B : {2 * G.M, 2 * G.N}) {
      if (s != SG_OK) break;
      if (!roots64.count(B)) {
        void* d = nullptr;
        s = upload_roots<double>(p, B, &d);
        roots64[B] = d;
      }
      if (s == SG_OK && !p->roots.count(B)) {
        void* d = nullptr;
        s = prec == SG_FP64 ? SG_OK : upload_roots<float>(p, B, &d);
        p->roots[B] = prec == SG_FP64 ? roots64[B] : d;
      }
    }
    if (s == SG_OK) {
      G.r2m = p->roots[2 * G.M];
      G.r2n = p->roots[2 * G.N];
      const int pc = prec == SG_FP64 ? 0 : 1;
      void** slots[3] = {&G.twA, &G.twB, &G.twC};
      for (int pass = 0; pass < 3 && s == SG_OK; ++pass) {
        const int len = pass == 1 ? G.N : G.M;
        const auto tk = std::make_pair(pass, len);
        if (!tw.count(tk)) {
          void* d = nullptr;
          s = make_twiddles(p, pc, pass, len, pass == 1 ? G.r2n : G.r2m, &d);
          tw[tk] = d;
        }
        *slots[pass] = tw[tk];
      }
      // inverse rows in launch variant 1 (pass code 4), where it exists
      if (s == SG_OK && sg_variants(pc, 2, G.M) > 1) {
        const auto tk = std::make_pair(4, G.M);
        if (!tw.count(tk)) {
          void* d = nullptr;
          s = make_twiddles(p, pc, 4, G.M, G.r2m, &d);
          tw[tk] = d;
        }
        G.twC1 = tw[tk];
      }
      if (s == SG_OK && G.fs) {
        if (!twfs.count(G.N)) {
          void* d = nullptr;
          s = upload_fs_twiddles(p, pc, G.N, &d);
          twfs[G.N] = d;
        }
        G.twfs = twfs[G.N];
      }
      if (s == SG_OK && fresh) s = build_spectra(p, G, roots64[2 * G.M], roots64[2 * G.N]);
    }
    p->grids.push_back(G);
  }
  p->total = off;
  // classes of equal (nx, ny, order), in order of first appearance, with
  // their device descriptors
  for (int i = 0; i < (int)p->grids.size() && s == SG_OK; ++i) {
    const GridPlan& G = p->grids[i];
    GridClass* c = nullptr;
    for (GridClass& x : p->classes)
      if (x.M == G.M && x.N == G.N && x.k == G.k) c = &x;
    if (!c) {
      GridClass nc;
      nc.M = G.M;
      nc.N = G.N;
      nc.k = G.k;
      const int pc = prec == SG_FP64 ? 0 : 1;
      // the Stockham column pass has variants; the four-step one has none
      nc.var[1] = G.fs ? 0 : sg_default_variant(pc, 1, G.N);
      nc.var[2] = sg_default_variant(pc, 2, G.M);
      p->classes.push_back(nc);
      c = &p->classes.back();
    }
    c->members.push_back(i);
  }
  for (GridClass& c : p->classes) {
    if (s != SG_OK) break;
    std::vector<sg_bgrid> h(c.members.size());
    for (size_t j = 0; j < c.members.size(); ++j) {
      const GridPlan& G = p->grids[c.members[j]];
      h[j] = sg_bgrid{G.off, G.X, G.V, G.tabx, G.taby};
    }
    s = dev_alloc(p, (void**)&c.desc, h.size() * sizeof(sg_bgrid));
    if (s == SG_OK)
      s = hip_check(p, hipMemcpy(c.desc, h.data(), h.size() * sizeof(sg_bgrid), hipMemcpyHostToDevice),
                    "descriptor upload");
    for (sg_bgrid& d : h) d.X = d.V;
    if (s == SG_OK) s = dev_alloc(p, (void**)&c.desc_y, h.size() * sizeof(sg_bgrid));
    if (s == SG_OK)
      s = hip_check(p, hipMemcpy(c.desc_y, h.data(), h.size() * sizeof(sg_bgrid), hipMemcpyHostToDevice),
                    "descriptor upload");
  }
  // the no-allocation variant: every grid's X and V laid out in scratch
  // (256-byte aligned), with descriptors of their own
  if (s == SG_OK) {
    const size_t cb = prec == SG_FP64 ? 16 : 8;
    std::vector<int64_t> xo(p->grids.size()), vo(p->grids.size());
    int64_t at = 0;
    for (size_t i = 0; i < p->grids.size(); ++i) {
      const GridPlan& G = p->grids[i];
      xo[i] = at;
      at += ((int64_t)(cb * (size_t)G.M * G.N) + 255) / 256 * 256;
      vo[i] = at;
      at += ((int64_t)(cb * 2 * (size_t)G.M * G.N) + 255) / 256 * 256;
    }
    p->noalloc_bytes = at;
    p->noalloc_ok = at <= (int64_t)SG_NOALLOC_BYTES;
    void* base = nullptr;
    if (p->noalloc_ok) {
      hipError_t e = scratch_address(p->device, &base);
      if (e != hipSuccess) s = hip_check(p, e, "hipGetSymbolAddress(scratch)");
    }
    for (GridClass& c : p->classes) {
      if (s != SG_OK || !p->noalloc_ok) break;
      std::vector<sg_bgrid> h(c.members.size());
      for (size_t j = 0; j < c.members.size(); ++j) {
        const int gi = c.members[j];
        const GridPlan& G = p->grids[gi];
        h[j] = sg_bgrid{G.off, (char*)base + xo[gi], (char*)base + vo[gi], G.tabx, G.taby};
      }
      s = dev_alloc(p, (void**)&c.desc_s, h.size() * sizeof(sg_bgrid));
      if (s == SG_OK)
        s = hip_check(p, hipMemcpy(c.desc_s, h.data(), h.size() * sizeof(sg_bgrid), hipMemcpyHostToDevice),
                      "descriptor upload");
    }
  }
  if (s == SG_OK && (flags & SG_FLAG_GRAPH)) {
    const int nside = std::min<int>(kSideStreams, (int)p->classes.size());
    for (int i = 0; i < nside && s == SG_OK; ++i) {
      hipStream_t q = nullptr;
      hipEvent_t ev = nullptr;
      if (hipStreamCreateWithFlags(&q, hipStreamNonBlocking) != hipSuccess)
        s = fail(SG_ERR_DEVICE, "hipStreamCreateWithFlags");
      else
        p->side.push_back(q);
      if (s == SG_OK && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
        s = fail(SG_ERR_DEVICE, "hipEventCreateWithFlags");
      else if (s == SG_OK)
        p->sync_ev.push_back(ev);
    }
    // two more: the caller's stream -> side stream 0, and back
    for (int i = 0; i < 2 && s == SG_OK; ++i) {
      hipEvent_t ev = nullptr;
      if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
        s = fail(SG_ERR_DEVICE, "hipEventCreateWithFlags");
      else
        p->sync_ev.push_back(ev);
    }
  }
  if (s == SG_OK) s = tune(p);
  if (s == SG_OK) s = dev_alloc(p, (void**)&p->flag, sizeof(int));
  if (s != SG_OK) {
    std::string keep = g_msg;
    (void)hipStreamSynchronize(p->st);
    release(p);
    delete p;
    g_msg = keep;
    return s;
  }
  if (env_on("SG_LOG")) {
    fprintf(stderr, "sg: plan %p: %d grids, %s, %lld device bytes, %zu classes\n", (void*)p, (int)p->grids.size(),
            prec == SG_FP64 ? "FP64" : "FP32-split", (long long)p->bytes, p->classes.size());
    static const char* src[3] = {"defaults", "timed", "stored"};
    for (const GridClass& c : p->classes) {
      const GridPlan& G = p->grids[c.members[0]];
      fprintf(stderr,
              "sg:   %dx%d k=%d grids=%zu: columns %s, variants %d/%d/%d, tiles %d/%d/%d (%s), spectra %d B per bin\n",
              c.M, c.N, c.k, c.members.size(), G.fs ? "four-step" : "Stockham", c.var[0], c.var[1], c.var[2], c.tile[0],
              c.tile[1], c.tile[2], src[c.src], G.tab_bytes);
    }
  }
  *out = p;
  return SG_OK;
}

sg_status sg_plan_destroy(sg_plan p) {
  g_msg.clear();
  if (!p) return SG_OK;
  (void)hipStreamSynchronize(p->st);
  release(p);
  delete p;
  return SG_OK;
}

sg_status sg_plan_layout(sg_plan p, int64_t* offsets) {
  g_msg.clear();
  if (!p) return fail(SG_ERR_ARG, "plan is NULL");
  if (!offsets) return fail(SG_ERR_ARG, "offsets is NULL");
  for (size_t i = 0; i < p->grids.size(); ++i) offsets[i] = p->grids[i].off;
  offsets[p->grids.size()] = p->total;
  return SG_OK;
}

sg_status sg_plan_info(sg_plan p, int32_t* ngrids, int32_t* prec, int64_t* device_bytes) {
  g_msg.clear();
  if (!p) return fail(SG_ERR_ARG, "plan is NULL");
  if (ngrids) *ngrids = (int32_t)p->grids.size();
  if (prec) *prec = (int32_t)p->prec;
  if (device_bytes) *device_bytes = p->bytes;
  return SG_OK;
}

sg_status sg_sample_points(sg_plan p, int32_t g, double* xs0, double* ys0, double* dx, double* dy) {
  g_msg.clear();
  if (!p) return fail(SG_ERR_ARG, "plan is NULL");
  if (g < 0 || g >= (int32_t)p->grids.size()) return fail(SG_ERR_ARG, "grid index %d out of range", g);
  const GridPlan& G = p->grids[g];
  const double off = (G.k % 2 == 1) ? 0.5 : 1.0;  // cell centres (odd k) or vertices x0 + (i+1) dx (even k)
  if (xs0) *xs0 = G.g.x0 + off * G.hx;
  if (ys0) *ys0 = G.g.y0 + off * G.hy;
  if (dx) *dx = G.hx;
  if (dy) *dy = G.hy;
  return SG_OK;
}

sg_status sg_weights(sg_plan p, int32_t g, double* wx, double* wy) {
  g_msg.clear();
  sg_status s = check_plan(p);
  if (s != SG_OK) return s;
  if (g < 0 || g >= (int32_t)p->grids.size()) return fail(SG_ERR_ARG, "grid index %d out of range", g);
  if (!wx && !wy) return SG_OK;
  const GridPlan& G = p->grids[g];
  return hip_check(p, sg_launch_weights(G.k, G.hx, G.hy, G.M, G.N, wx, wy, 1, p->st), "weights launch");
}

sg_status sg_bspline_coeffs(sg_plan p, const void* sigma, void* coeffs) {
  g_msg.clear();
  sg_status s = step_entry(p);
  if (s != SG_OK) return s;
  if (!sigma || !coeffs) return fail(SG_ERR_ARG, "sigma or coeffs is NULL");
  const int prec = p->prec == SG_FP64 ? 0 : 1;
  const size_t el = prec == 0 ? 8 : 4;
  for (const GridPlan& G : p->grids) {
    const char* src = (const char*)sigma + el * G.off;
    char* dst = (char*)coeffs + el * G.off;
    hipError_t e = hipSuccess;
    if (G.k >= 3) {
      e = sg_launch_coeff_rows(prec, G.M, src, dst, G.N, G.k, p->st);
      if (e == hipSuccess) e = sg_launch_coeff_cols(prec, G.N, dst, G.M, G.k, p->st);
    } else if (src != dst) {
      e = hipMemcpyAsync(dst, src, el * (size_t)G.M * G.N, hipMemcpyDeviceToDevice, p->st);
    }
    if (e != hipSuccess) return hip_check(p, e, "coefficient launch");
  }
  return SG_OK;
}

sg_status sg_forces(sg_plan p, const void* sigma, void* fx, void* fy) {
  g_msg.clear();
  Range range("sg_forces");
  sg_status s = step_entry(p);
  if (s != SG_OK) return s;
  if (!sigma || !fx || !fy) return fail(SG_ERR_ARG, "sigma, fx or fy is NULL");
  if (fx == fy || fx == sigma || fy == sigma) return fail(SG_ERR_ARG, "fx, fy and sigma must not alias");
  const int prec = p->prec == SG_FP64 ? 0 : 1;
  if (p->flags & SG_FLAG_CHECK_FINITE) {
    int h = 0;
    hipError_t e = hipMemsetAsync(p->flag, 0, sizeof(int), p->st);
    if (e == hipSuccess) e = sg_launch_check_finite(prec, sigma, p->total, p->flag, p->st);
    if (e == hipSuccess) e = hipMemcpyAsync(&h, p->flag, sizeof(int), hipMemcpyDeviceToHost, p->st);
    if (e == hipSuccess) e = hipStreamSynchronize(p->st);
    if (e != hipSuccess) return hip_check(p, e, "finite check");
    if (h) return fail(SG_ERR_STATE, "sigma holds NaN or Inf");
  }
  if (p->flags & SG_FLAG_GRAPH) {
    // replay the captured step for these buffers (capture it on first use),
    // ordered after the caller's stream and before its later work
    StepGraph* g = nullptr;
    for (size_t i = 0; i < p->graphs.size(); ++i)
      if (p->graphs[i].sigma == sigma && p->graphs[i].fx == fx && p->graphs[i].fy == fy) {
        std::rotate(p->graphs.begin(), p->graphs.begin() + i, p->graphs.begin() + i + 1);
        g = &p->graphs[0];
        break;
      }
    if (!g) {
      if (p->graphs.size() >= kMaxGraphs) {
        StepGraph& old = p->graphs.back();
        (void)hipGraphExecDestroy(old.exec);
        (void)hipGraphDestroy(old.graph);
        p->graphs.pop_back();
      }
      StepGraph ng;
      s = capture_step(p, sigma, fx, fy, &ng);
      if (s != SG_OK) return s;
      p->graphs.insert(p->graphs.begin(), ng);
      g = &p->graphs[0];
    }
    const size_t nside = p->side.size();
    hipEvent_t in = p->sync_ev[nside], out = p->sync_ev[nside + 1];
    hipError_t e = hipEventRecord(in, p->st);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->side[0], in, 0);
    if (e == hipSuccess) e = hipGraphLaunch(g->exec, p->side[0]);
    if (e == hipSuccess) e = hipEventRecord(out, p->side[0]);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->st, out, 0);
    if (e != hipSuccess) return hip_check(p, e, "graph launch");
    if (p->timing) ++p->timed_calls;
    return SG_OK;
  }
  for (const GridClass& c : p->classes) {
    // one launch per pass for every grid of the class, timing marks around them
    Range crange("class %dx%d k=%d", c.M, c.N, c.k);
    hipError_t e = mark(p);
    const GridPlan& G = p->grids[c.members[0]];
    const int solve = c.k >= 3 ? c.k : 0;
    const int ng = (int)c.members.size();
    const int tj = sg_row_tile(prec, c.M, c.N);
    if (e == hipSuccess)
      e = sg_launch_row_fwd(prec, c.M, sigma, c.M, nullptr, c.N, G.r2m, solve, 0, G.twA, c.desc, ng, c.tile[0], p->st);
    if (e == hipSuccess) e = mark(p);
    if (e == hipSuccess) e = launch_cols(p, c, c.tile[1], p->st);
    if (e == hipSuccess) e = mark(p);
    if (e == hipSuccess) e = launch_rows_inv(p, c, fx, fy, c.tile[2], p->st, c.desc);
    if (e == hipSuccess) e = mark(p);
    if (e != hipSuccess) return hip_check(p, e, "force launch");
  }
  if (p->timing) ++p->timed_calls;
  return SG_OK;
}

sg_status sg_forces_noalloc(sg_plan p, const void* sigma, void* fx, void* fy) {
  g_msg.clear();
  Range range("sg_forces_noalloc");
  sg_status s = step_entry(p);
  if (s != SG_OK) return s;
  if (!sigma || !fx || !fy) return fail(SG_ERR_ARG, "sigma, fx or fy is NULL");
  if (fx == fy || fx == sigma || fy == sigma) return fail(SG_ERR_ARG, "fx, fy and sigma must not alias");
  if (!p->noalloc_ok)
    return fail(SG_ERR_ARG, "the plan's workspace (%lld bytes) exceeds the %llu-byte no-allocation scratch",
                (long long)p->noalloc_bytes, (unsigned long long)SG_NOALLOC_BYTES);
  const int prec = p->prec == SG_FP64 ? 0 : 1;
  // the same launches as sg_forces (eager, on the plan's stream), with X and
  // V in scratch; nothing is allocated, cleared or synchronised
  for (const GridClass& c : p->classes) {
    const GridPlan& G = p->grids[c.members[0]];
    const int solve = c.k >= 3 ? c.k : 0;
    const int ng = (int)c.members.size();
    const int tj = sg_row_tile(prec, c.M, c.N);
    hipError_t e = sg_launch_row_fwd(prec, c.M, sigma, c.M, nullptr, c.N, G.r2m, solve, 0, G.twA, c.desc_s, ng,
                                     c.tile[0], p->st);
    if (e == hipSuccess) e = launch_cols(p, c, c.tile[1], p->st, c.desc_s);
    if (e == hipSuccess) e = launch_rows_inv(p, c, fx, fy, c.tile[2], p->st, c.desc_s);
    if (e != hipSuccess) return hip_check(p, e, "force launch (no allocation)");
  }
  return SG_OK;
}

sg_status sg_plan_classes(sg_plan p, int32_t* nclasses, int32_t* info, int32_t cap) {
  g_msg.clear();
  if (!p) return fail(SG_ERR_ARG, "plan is NULL");
  if (nclasses) *nclasses = (int32_t)p->classes.size();
  if (info) {
    const int prec = p->prec == SG_FP64 ? 0 : 1;
    for (int32_t i = 0; i < cap && i < (int32_t)p->classes.size(); ++i) {
      const GridClass& c = p->classes[i];
      int32_t* o = info + 8 * i;
      o[0] = c.M;
      o[1] = c.N;
      o[2] = c.k;
      o[3] = (int32_t)c.members.size();
      for (int pass = 0; pass < 3; ++pass) {
        // the tile the launch uses: rows capped by the row count; columns the
        // largest power of two that divides nx
        int t = c.tile[pass] > 0 ? c.tile[pass] : sg_max_tile(prec, pass, pass == 1 ? c.N : c.M, c.var[pass]);
        if (pass == 1) {
          int d = 1;
          while (d < t && c.M % (2 * d) == 0) d *= 2;
          t = d;
        } else if (t > c.N) {
          t = c.N;
        }
        o[4 + pass] = t;
      }
      o[7] = c.src;
    }
  }
  return SG_OK;
}

sg_status sg_plan_tuning(sg_plan p, int32_t cls, int32_t* out) {
  g_msg.clear();
  if (!p) return fail(SG_ERR_ARG, "plan is NULL");
  if (!out) return fail(SG_ERR_ARG, "out is NULL");
  if (cls < 0 || cls >= (int32_t)p->classes.size()) return fail(SG_ERR_ARG, "class %d out of range", (int)cls);
  const GridClass& c = p->classes[cls];
  for (int pass = 0; pass < 3; ++pass) {
    out[pass] = c.var[pass];
    out[3 + pass] = c.tile[pass];
  }
  out[6] = c.src;
  out[7] = 0;
  return SG_OK;
}

sg_status sg_plan_set_timing(sg_plan p, int32_t enable) {
  g_msg.clear();
  sg_status s = check_plan(p);
  if (s != SG_OK) return s;
  hipError_t e = hipStreamSynchronize(p->st);
  if (e != hipSuccess) return hip_check(p, e, "timing sync");
  drop_events(p);
  p->timing = enable != 0;
  return SG_OK;
}

sg_status sg_plan_pass_times(sg_plan p, double* ms, int64_t* calls) {
  g_msg.clear();
  sg_status s = check_plan(p);
  if (s != SG_OK) return s;
  if (!ms) return fail(SG_ERR_ARG, "ms is NULL");
  hipError_t e = hipStreamSynchronize(p->st);
  if (e != hipSuccess) return hip_check(p, e, "timing sync");
  ms[0] = ms[1] = ms[2] = 0.0;
  for (size_t i = 0; i + 3 < p->ev.size(); i += 4)
    for (int k = 0; k < 3; ++k) {
      float t = 0.0f;
      e = hipEventElapsedTime(&t, p->ev[i + k], p->ev[i + k + 1]);
      if (e != hipSuccess) return hip_check(p, e, "hipEventElapsedTime");
      ms[k] += (double)t;
    }
  if (calls) *calls = p->timed_calls;
  drop_events(p);
  return SG_OK;
}

sg_status sg_forces_adjoint(sg_plan p, const void* gfx, const void* gfy, void* gsigma) {
  Range range("sg_forces_adjoint");
  g_msg.clear();
  sg_status s = step_entry(p);
  if (s != SG_OK) return s;
  if (!gfx || !gfy || !gsigma) return fail(SG_ERR_ARG, "gfx, gfy or gsigma is NULL");
  if (gsigma == gfx || gsigma == gfy) return fail(SG_ERR_ARG, "gsigma must not alias gfx or gfy");
  const int prec = p->prec == SG_FP64 ? 0 : 1;
  // per class, all grids at once: row spectra of gx in X, of gy in the first
  // half of V (descriptors desc_y), gC spectra in its second half
  for (const GridClass& c : p->classes) {
    const GridPlan& G = p->grids[c.members[0]];
    const int solve = c.k >= 3 ? c.k : 0;
    const int ng = (int)c.members.size();
    const int tj = sg_row_tile(prec, c.M, c.N);
    hipError_t e =
        sg_launch_row_fwd(prec, c.M, gfx, c.M, nullptr, c.N, G.r2m, 0, 0, G.twA, c.desc, ng, c.tile[0], p->st);
    if (e == hipSuccess)
      e = sg_launch_row_fwd(prec, c.M, gfy, c.M, nullptr, c.N, G.r2m, 0, 0, G.twA, c.desc_y, ng, c.tile[0], p->st);
    if (e == hipSuccess && G.fs_adj) {
      e = sg_launch_colfs_adj(prec, c.N, nullptr, nullptr, nullptr, c.M, tj, nullptr, nullptr, G.kind, G.tab_bytes, G.r2n,
                              solve, G.twfs, c.desc, ng, p->st);
      if (e == hipSuccess)
        e = sg_launch_row_c2r(prec, c.M, c.N, nullptr, gsigma, tj, G.r2m, solve, G.twA, c.desc, ng, p->st);
    } else if (e == hipSuccess) {
      e = sg_launch_adjoint_tail(prec, c.M, c.N, nullptr, nullptr, nullptr, gsigma, tj, nullptr, nullptr, G.kind, G.r2m,
                                 G.r2n, solve, G.twB, G.twA, c.desc, ng, p->st);
    }
    if (e != hipSuccess) return hip_check(p, e, "adjoint launch");
  }
  return SG_OK;
}

}  // extern "C"
