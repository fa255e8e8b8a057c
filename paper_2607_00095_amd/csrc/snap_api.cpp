// Host side of the C ABI declared in include/snap.h: plan construction
// (shapes, groupings, workspace layout; the sparsity structure is fixed once,
// as the paper exploits for repeated factorizations, Sec. III-B/III-C), and
// stream-ordered launches of the family kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "snap.h"
#include "snap_device.hpp"

namespace snap {
int slab_class(int nx, int nt);
int slab_launch(const KernelArgs& a, int cls, bool mixed, hipStream_t st);
int band_class(int nx, int nt, bool mixed);
int band_launch(const KernelArgs& a, int cls, bool mixed, hipStream_t st);
size_t band_workspace_bytes(int nx, int nt, bool mixed);
int slab_variants(int nx, int nt, int* out, int cap);
int band_variants(int nx, int nt, bool mixed, int* out, int cap);
int slab_waves(int cls);
int band_waves(int cls);
int band_sides(int cls);
int band_group_class(int cls, int min_nb, int count, int ncu);
bool spec_supported(int nx, int ny, int nt);
size_t spec_workspace_bytes(int nx, int nt);
int spec_launch(const KernelArgs& a, hipStream_t st);
bool bc_supported(int nx, int ny, int nt);
int bc_class(int nx);
int bc_launch(const KernelArgs& a, int cls, hipStream_t st);
}  // namespace snap

using namespace snap;

// Scratch for snap_project_noalloc: the workspace of callers that cannot
// allocate device memory.  Every GPU the library runs on holds its own copy
// until the process ends; its device address is looked up once per device at
// plan creation (the array's name in host code is only a host-side stand-in).
constexpr size_t kStaticScratchBytes = (size_t)SNAP_NOALLOC_MAX_WORKSPACE;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (0 on failure)
int scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return SNAP_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return SNAP_SUCCESS;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return SNAP_EHIP;
  }
  g_scratch_ptr[device] = ptr;
  return SNAP_SUCCESS;
}

void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

// Samples sharing one kernel instantiation (shapes may differ: every kernel
// reads its sample's shape from the descriptor).  `kind` 0 = slab rows,
// 1 = banded, 2 = spectral (2D diffusion + energy), 3 = boundary rows (Burgers
// boundary conditions + mass); `cls` = instantiation index; ids sorted by
// decreasing cost so the longest samples start first.
struct Group {
  int kind, cls;
  double cost = 0.0;
  std::vector<int32_t> ids;
  int32_t* d_ids = nullptr;
};

constexpr int kStreams = 4;   // groups are spread over this many internal streams
constexpr int kTimerEvents = 32768;  // event pool of the kernel timer

// A captured launch sequence and the call arguments it was captured with.
struct GraphSlot {
  hipGraphExec_t exec = nullptr;
  KernelArgs key{};
};

}  // namespace

struct snap_plan_s {
  int32_t batch = 0;
  snap_options opt{};
  std::vector<snap_sample_desc> descs;
  snap_sample_desc* d_descs = nullptr;
  std::vector<Group> groups;
  std::vector<int64_t> ws_off;   // per-sample byte offsets
  int64_t* d_ws_off = nullptr;
  double* d_tab = nullptr;              // Fourier basis tables (2D family)
  size_t ws_bytes = 0;
  int64_t total_vars = 0, total_rows = 0, total_aux = 0;
  int device = 0;
  std::vector<hipStream_t> streams;     // fork/join of independent groups
  std::vector<hipEvent_t> events;       // [0] fork, [1..] join per stream
  GraphSlot graphs[2];                  // SNAP_FLAG_GRAPH: forward, backward
  std::mutex graph_mu;
  KernelTimer* timer = nullptr;         // snap_plan_set_kernel_timing
  std::mutex run_mu;                    // calls on one plan from several threads
};

namespace snap {
// Events recorded around timed launches, in pairs per launch: (kernel id,
// pool index) in recording order.  Marks past the pool's end are dropped and
// counted.
struct KernelTimer {
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, int>> marks;
  int64_t dropped = 0;
};
thread_local KernelTimer* tl_timer = nullptr;

void timer_mark(KernelTimer* t, int kernel, hipStream_t st) {
  if (t->marks.size() >= t->pool.size()) { ++t->dropped; return; }
  const int i = (int)t->marks.size();
  if (hipEventRecord(t->pool[i], st) == hipSuccess) t->marks.emplace_back(kernel, i);
}
}  // namespace snap

namespace {

int64_t rows_of(const snap_sample_desc& d) {
  switch (d.family) {
    case SNAP_MASS_IC:
    case SNAP_FISHER_KPP: return (int64_t)d.nx + d.nt - 1;
    case SNAP_BURGERS_LF:
    case SNAP_BURGERS_GODUNOV: return (int64_t)d.nx * (d.nt - 1);
    case SNAP_DIFF2D_ENERGY: return (int64_t)d.nx * d.ny * (d.nt - 1) + d.nt;
    case SNAP_BURGERS_BC: return 3 * (int64_t)d.nt;
    default: return -1;
  }
}

int64_t aux_of(const snap_sample_desc& d) {
  switch (d.family) {
    case SNAP_MASS_IC: return d.nx + 1;
    case SNAP_FISHER_KPP: return d.nx;
    case SNAP_DIFF2D_ENERGY: return d.nt;
    case SNAP_BURGERS_BC: return 2;
    default: return 0;
  }
}

void free_timer(snap_plan p) {
  if (!p->timer) return;
  for (auto& e : p->timer->pool) (void)hipEventDestroy(e);
  delete p->timer;
  p->timer = nullptr;
}

void free_plan(snap_plan p) {
  if (!p) return;
  free_timer(p);
  for (auto& g : p->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  for (auto& e : p->events) (void)hipEventDestroy(e);
  for (auto& s : p->streams) (void)hipStreamDestroy(s);
  for (auto& g : p->groups)
    if (g.d_ids) (void)hipFree(g.d_ids);
  if (p->d_descs) (void)hipFree(p->d_descs);
  if (p->d_ws_off) (void)hipFree(p->d_ws_off);
  if (p->d_tab) (void)hipFree(p->d_tab);
  delete p;
}

bool options_valid(const snap_options& o) {
  return o.tol_h > 0 && o.tol_s > 0 && o.max_newton >= 1 && o.max_ls >= 0 &&
         (o.precision == SNAP_PREC_FP64 || o.precision == SNAP_PREC_MIXED);
}

// ---------------------------------------------------------------- autotuner
// SNAP_FLAG_AUTOTUNE: for every group with more than one buildable launch
// shape, time each on a synthetic copy of the group (same shapes, same sample
// count, seeded smooth fields plus noise, two Newton iterations) and keep the
// fastest.  Choices are cached per process by group signature.

// candidate classes common to every sample of a group
std::vector<int> group_candidates(const snap_plan_s& p, const Group& g) {
  std::vector<int> cand;
  for (size_t i = 0; i < g.ids.size(); ++i) {
    const snap_sample_desc& d = p.descs[g.ids[i]];
    int v[8];
    const int n = g.kind == 0 ? slab_variants(d.nx, d.nt, v, 8)
                  : g.kind == 1 ? band_variants(d.nx, d.nt, p.opt.precision == SNAP_PREC_MIXED, v, 8)
                                : (v[0] = 0, 1);
    std::vector<int> mine(v, v + n);
    if (i == 0) {
      cand = mine;
    } else {
      std::vector<int> keep;
      for (int c : cand)
        if (std::find(mine.begin(), mine.end(), c) != mine.end()) keep.push_back(c);
      cand = keep;
    }
  }
  return cand;
}

std::string group_signature(const snap_plan_s& p, const Group& g) {
  std::string k = std::to_string(g.kind) + ":" + std::to_string(g.cls) + ":" +
                  std::to_string(p.opt.precision) + ":" + std::to_string(g.ids.size());
  for (int32_t id : g.ids) {
    const snap_sample_desc& d = p.descs[id];
    k += ":" + std::to_string(d.family) + "," + std::to_string(d.nx) + "," + std::to_string(d.nt);
  }
  return k;
}

std::mutex g_tune_mu;
std::map<std::string, int> g_tune_cache;

// deterministic pseudo-random numbers in [-0.5, 0.5) (64-bit LCG)
struct Lcg {
  uint64_t s;
  double next() {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(s >> 11) * (1.0 / 9007199254740992.0) - 0.5;
  }
};

int64_t rows_of(const snap_sample_desc& d);
int64_t aux_of(const snap_sample_desc& d);
int launch_group_cls(const snap_plan_s& p, KernelArgs a, const Group& g, int cls, hipStream_t st);

// Time the candidates; returns the fastest class (or the group's own class
// if anything fails: tuning never changes results, only launch shapes).
int tune_group(const snap_plan_s& p, const Group& g, const std::vector<int>& cand,
               size_t (*ws_need)(const snap_sample_desc&, bool)) {
  const bool mixed = p.opt.precision == SNAP_PREC_MIXED;
  const int n = (int)g.ids.size();
  std::vector<snap_sample_desc> d(n);
  std::vector<int64_t> off(n);
  std::vector<int32_t> order(n);
  int64_t nv = 0, nr = 0, na = 0;
  size_t ws = 0;
  for (int i = 0; i < n; ++i) {
    d[i] = p.descs[g.ids[i]];
    d[i].var_off = nv; d[i].row_off = nr; d[i].aux_off = na;
    nv += (int64_t)d[i].nx * d[i].nt; nr += rows_of(d[i]); na += aux_of(d[i]);
    off[i] = (int64_t)ws;
    ws += (ws_need(d[i], mixed) + 255) & ~(size_t)255;
    order[i] = i;
  }
  // seeded fields: smooth profile plus noise, aux from the t = 0 slab
  std::vector<double> uh((size_t)nv), aux((size_t)std::max<int64_t>(na, 1), 0.0);
  Lcg rng{0x5eed5eedull};
  for (int i = 0; i < n; ++i) {
    const snap_sample_desc& q = d[i];
    const bool burgers = q.family == SNAP_BURGERS_LF || q.family == SNAP_BURGERS_GODUNOV;
    for (int k = 0; k < q.nt; ++k)
      for (int x = 0; x < q.nx; ++x) {
        const double t = 6.283185307179586 * x / q.nx;
        const double base = burgers ? 0.5 * std::sin(t) : 0.5 + 0.3 * std::sin(t);
        uh[q.var_off + (int64_t)k * q.nx + x] = base + 0.02 * rng.next();
      }
    if (q.family == SNAP_MASS_IC || q.family == SNAP_FISHER_KPP) {
      double m0 = 0.0;
      for (int x = 0; x < q.nx; ++x) {
        const double t = 6.283185307179586 * x / q.nx;
        aux[q.aux_off + x] = 0.5 + 0.3 * std::sin(t);
        m0 += aux[q.aux_off + x];
      }
      if (q.family == SNAP_MASS_IC) aux[q.aux_off + q.nx] = m0;
    }
  }
  void *dd = nullptr, *dord = nullptr, *doff = nullptr, *duh = nullptr, *daux = nullptr,
       *du = nullptr, *dlam = nullptr, *dst = nullptr, *dws = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipStream_t st = nullptr;
  int best = g.cls;
  bool ok = hipMalloc(&dd, sizeof(snap_sample_desc) * n) == hipSuccess &&
            hipMalloc(&dord, sizeof(int32_t) * n) == hipSuccess &&
            hipMalloc(&doff, sizeof(int64_t) * n) == hipSuccess &&
            hipMalloc(&duh, sizeof(double) * nv) == hipSuccess &&
            hipMalloc(&daux, sizeof(double) * aux.size()) == hipSuccess &&
            hipMalloc(&du, sizeof(double) * nv) == hipSuccess &&
            hipMalloc(&dlam, sizeof(double) * std::max<int64_t>(nr, 1)) == hipSuccess &&
            hipMalloc(&dst, sizeof(snap_sample_stats) * n) == hipSuccess &&
            hipMalloc(&dws, std::max<size_t>(ws, 256)) == hipSuccess &&
            hipMemcpy(dd, d.data(), sizeof(snap_sample_desc) * n, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(dord, order.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(doff, off.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(duh, uh.data(), sizeof(double) * nv, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(daux, aux.data(), sizeof(double) * aux.size(), hipMemcpyHostToDevice) == hipSuccess &&
            hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
  if (ok) {
    KernelArgs a{};
    a.descs = (const snap_sample_desc*)dd;
    a.uhat = (const double*)duh;
    a.aux = (const double*)daux;
    a.u = (double*)du;
    a.lam = (double*)dlam;
    a.stats = (snap_sample_stats*)dst;
    a.ws = (unsigned char*)dws;
    a.ws_off = (const int64_t*)doff;
    a.opt = p.opt;
    a.opt.max_newton = 2;
    a.opt.flags = 0;
    a.backward = 0;
    Group tg = g;
    tg.d_ids = (int32_t*)dord;
    float best_ms = 0.0f;
    for (int c : cand) {
      float ms_min = -1.0f;
      for (int rep = 0; rep < 3 && ok; ++rep) {   // first run warms up
        ok = hipEventRecord(e0, st) == hipSuccess && launch_group_cls(p, a, tg, c, st) == 0 &&
             hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.0f;
        if (ok && rep > 0 && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
          ms_min = ms_min < 0.0f ? ms : std::min(ms_min, ms);
      }
      if (!ok) break;
      if (ms_min >= 0.0f && (best_ms == 0.0f || ms_min < best_ms)) { best_ms = ms_min; best = c; }
    }
  }
  if (!ok) best = g.cls;
  if (st) (void)hipStreamSynchronize(st);
  for (void* q : {dd, dord, doff, duh, daux, du, dlam, dst, dws})
    if (q) (void)hipFree(q);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st) (void)hipStreamDestroy(st);
  (void)hipGetLastError();
  return best;
}

size_t slab_ws_need(const snap_sample_desc&, bool) { return 0; }
size_t band_ws_need(const snap_sample_desc& d, bool mixed) { return band_workspace_bytes(d.nx, d.nt, mixed); }

}  // namespace

extern "C" {

void snap_default_options(snap_options* opt) {
  if (!opt) return;
  opt->tol_h = 1e-11;
  opt->tol_s = 1e-11;
  opt->max_newton = 20;
  opt->max_ls = 30;
  opt->precision = SNAP_PREC_FP64;
  opt->flags = 0;
}

int snap_plan_create(snap_plan* out, int32_t batch, const snap_sample_desc* descs_host,
                     const snap_options* opt) {
  if (!out || batch < 0 || (batch > 0 && !descs_host)) return SNAP_EINVAL;
  *out = nullptr;
  snap_options o;
  if (opt) o = *opt; else snap_default_options(&o);
  if (!options_valid(o)) return SNAP_EINVAL;
  const bool mixed = o.precision == SNAP_PREC_MIXED;

  snap_plan p = new (std::nothrow) snap_plan_s();
  if (!p) return SNAP_ENOMEM;
  p->batch = batch;
  p->opt = o;
  p->descs.assign(descs_host, descs_host + batch);
  if (hipGetDevice(&p->device) != hipSuccess) { free_plan(p); return SNAP_EHIP; }

  std::map<std::pair<int, int>, size_t> gidx;
  std::vector<double> cost(batch, 0.0);
  p->ws_off.assign(batch, 0);
  size_t ws = 0;
  for (int32_t s = 0; s < batch; ++s) {
    const snap_sample_desc& d = p->descs[s];
    if (d.nx < 1 || d.nt < 1 || d.ny < 1 || d.var_off < 0 || d.row_off < 0 || d.aux_off < 0 ||
        (d.ny != 1 && d.family != SNAP_DIFF2D_ENERGY)) {
      free_plan(p); return SNAP_EINVAL;
    }
    const int64_t m = rows_of(d);
    if (m < 0) { free_plan(p); return SNAP_EUNSUPPORTED; }
    int kind = -1, cls = -1;
    size_t need = 0;
    if (d.family == SNAP_MASS_IC || d.family == SNAP_FISHER_KPP) {
      kind = 0;
      cls = slab_class(d.nx, d.nt);
      if (d.family == SNAP_FISHER_KPP && !(d.dt > 0.0)) cls = -1;
      cost[s] = (double)d.nx * d.nt;
    } else if (d.family == SNAP_BURGERS_LF || d.family == SNAP_BURGERS_GODUNOV) {
      kind = 1;
      cls = (d.dt > 0.0 && d.dx > 0.0) ? band_class(d.nx, d.nt, mixed) : -1;
      if (cls > 0) need = band_workspace_bytes(d.nx, d.nt, mixed);
      // factorization work ~ rows x (block bandwidth)^2
      cost[s] = (double)d.nx * (d.nt - 1) * (double)(cls % 32 + 1) * (cls % 32 + 1) * 256.0;
    } else if (d.family == SNAP_DIFF2D_ENERGY) {
      kind = 2;
      cls = (d.dt > 0.0 && d.dx > 0.0 && d.p0 >= 0.0 && spec_supported(d.nx, d.ny, d.nt)) ? 0 : -1;
      if (cls == 0) need = spec_workspace_bytes(d.nx, d.nt);
      cost[s] = (double)d.nx * d.ny * 16.0 * 40.0;
    } else if (d.family == SNAP_BURGERS_BC) {
      kind = 3;
      cls = (d.dx > 0.0 && bc_supported(d.nx, d.ny, d.nt)) ? bc_class(d.nx) : -1;
      cost[s] = (double)d.nx * d.nt;
    }
    if (cls < 0) { free_plan(p); return SNAP_EUNSUPPORTED; }
    p->ws_off[s] = (int64_t)ws;
    ws += (need + 255) & ~(size_t)255;
    const int64_t nvar = (int64_t)d.nx * d.ny * d.nt;
    p->total_vars = std::max(p->total_vars, d.var_off + nvar);
    p->total_rows = std::max(p->total_rows, d.row_off + m);
    p->total_aux = std::max(p->total_aux, d.aux_off + aux_of(d));
    auto key = std::make_pair(kind, cls);
    auto it = gidx.find(key);
    size_t gi;
    if (it == gidx.end()) {
      gi = p->groups.size();
      gidx[key] = gi;
      Group g;
      g.kind = kind;
      g.cls = cls;
      p->groups.push_back(g);
    } else {
      gi = it->second;
    }
    p->groups[gi].ids.push_back(s);
    p->groups[gi].cost += cost[s];
  }
  p->ws_bytes = std::max<size_t>(ws, 256);
  // banded groups smaller than the machine: the launch shape by group size
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess) {
    free_plan(p);
    return SNAP_EHIP;
  }
  for (auto& g : p->groups) {
    if (g.kind != 1) continue;
    int min_nb = INT32_MAX;
    for (int32_t id : g.ids) {
      const snap_sample_desc& d = p->descs[id];
      min_nb = std::min<int>(min_nb, (int)(((int64_t)d.nx * (d.nt - 1) + 15) / 16));
    }
    g.cls = band_group_class(g.cls, min_nb, (int)g.ids.size(), ncu);
  }
  // longest samples first inside a group; most expensive groups first
  for (auto& g : p->groups)
    std::stable_sort(g.ids.begin(), g.ids.end(),
                     [&](int32_t x, int32_t y) { return cost[x] > cost[y]; });
  std::stable_sort(p->groups.begin(), p->groups.end(),
                   [](const Group& x, const Group& y) { return x.cost > y.cost; });
  if (p->groups.size() > 1) {
    const int ns = std::min<int>(kStreams, (int)p->groups.size());
    p->events.resize(ns + 1, nullptr);
    for (auto& e : p->events)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) { free_plan(p); return SNAP_EHIP; }
    p->streams.resize(ns, nullptr);
    for (auto& st : p->streams)
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) { free_plan(p); return SNAP_EHIP; }
  }

  bool spectral = false;
  for (const auto& g : p->groups) spectral |= g.kind == 2;
  if (spectral) {
    // orthonormal real Fourier bases Q[x][j] and s_j = sin^2(pi f_j / N) for
    // N = 16, 32, 48, 64, packed as the kernel expects
    std::vector<double> tab;
    for (int n : {16, 32, 48, 64}) {
      const int half = n / 2;
      const double pi = 3.14159265358979323846;
      std::vector<double> q((size_t)n * n), s2(n);
      for (int x = 0; x < n; ++x)
        for (int j = 0; j < n; ++j) {
          double v;
          if (j == 0) v = 1.0 / std::sqrt((double)n);
          else if (j == half) v = (x % 2 ? -1.0 : 1.0) / std::sqrt((double)n);
          else {
            const int k = j < half ? j : j - half;
            const double ang = 2.0 * pi * (double)((k * x) % n) / n;
            v = std::sqrt(2.0 / n) * (j < half ? std::cos(ang) : std::sin(ang));
          }
          q[(size_t)x * n + j] = v;
        }
      for (int j = 0; j < n; ++j) {
        const int f = j <= half ? j : j - half;
        const double sn = std::sin(pi * f / n);
        s2[j] = sn * sn;
      }
      tab.insert(tab.end(), q.begin(), q.end());
      tab.insert(tab.end(), s2.begin(), s2.end());
    }
    if (hipMalloc(&p->d_tab, sizeof(double) * tab.size()) != hipSuccess ||
        hipMemcpy(p->d_tab, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice) != hipSuccess) {
      free_plan(p); return SNAP_ENOMEM;
    }
  }

  if (batch > 0) {
    if (hipMalloc(&p->d_descs, sizeof(snap_sample_desc) * batch) != hipSuccess ||
        hipMemcpy(p->d_descs, p->descs.data(), sizeof(snap_sample_desc) * batch,
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMalloc(&p->d_ws_off, sizeof(int64_t) * batch) != hipSuccess ||
        hipMemcpy(p->d_ws_off, p->ws_off.data(), sizeof(int64_t) * batch,
                  hipMemcpyHostToDevice) != hipSuccess) {
      free_plan(p); return SNAP_ENOMEM;
    }
    for (auto& g : p->groups) {
      if (hipMalloc(&g.d_ids, sizeof(int32_t) * g.ids.size()) != hipSuccess ||
          hipMemcpy(g.d_ids, g.ids.data(), sizeof(int32_t) * g.ids.size(),
                    hipMemcpyHostToDevice) != hipSuccess) {
        free_plan(p); return SNAP_ENOMEM;
      }
    }
  }
  // the no-allocation entry point's scratch: its address on this device
  // (set-up happens here, never on that entry point's own path)
  if (p->ws_bytes <= kStaticScratchBytes) (void)scratch_setup(p->device);
  if (o.flags & SNAP_FLAG_AUTOTUNE) {
    for (auto& g : p->groups) {
      const std::vector<int> cand = group_candidates(*p, g);
      if (cand.size() < 2) continue;
      const std::string key = group_signature(*p, g);
      std::lock_guard<std::mutex> lock(g_tune_mu);
      auto it = g_tune_cache.find(key);
      if (it != g_tune_cache.end()) {
        g.cls = it->second;
      } else {
        g.cls = tune_group(*p, g, cand, g.kind == 0 ? &slab_ws_need : &band_ws_need);
        g_tune_cache[key] = g.cls;
      }
    }
  }
  *out = p;
  return SNAP_SUCCESS;
}

int snap_plan_workspace_bytes(snap_plan plan, size_t* bytes) {
  if (!plan || !bytes) return SNAP_EINVAL;
  *bytes = plan->ws_bytes;
  return SNAP_SUCCESS;
}

int snap_plan_sizes(snap_plan plan, int64_t* total_vars, int64_t* total_rows, int64_t* total_aux) {
  if (!plan) return SNAP_EINVAL;
  if (total_vars) *total_vars = plan->total_vars;
  if (total_rows) *total_rows = plan->total_rows;
  if (total_aux) *total_aux = plan->total_aux;
  return SNAP_SUCCESS;
}

namespace {
int launch_group_cls(const snap_plan_s& p, KernelArgs a, const Group& g, int cls, hipStream_t st) {
  const bool mixed = p.opt.precision == SNAP_PREC_MIXED;
  a.order = g.d_ids;
  a.count = (int32_t)g.ids.size();
  a.tab = p.d_tab;
  if (g.kind == 2) return spec_launch(a, st);
  if (g.kind == 3) return bc_launch(a, cls, st);
  return g.kind == 0 ? slab_launch(a, cls, mixed, st) : band_launch(a, cls, mixed, st);
}
}  // namespace

static int launch_group(const snap_plan plan, KernelArgs a, const Group& g, hipStream_t st) {
  return launch_group_cls(*plan, a, g, g.cls, st);
}

// One group: launch on the caller's stream.  Several: fork onto the plan's
// streams (groups are independent), largest groups first, round robin, and
// join back so the caller's stream orders everything after the call.
static int run(snap_plan plan, KernelArgs a, hipStream_t st) {
  if (plan->groups.size() == 1) return launch_group(plan, a, plan->groups[0], st);
  const int ns = (int)plan->streams.size();
  if (hipEventRecord(plan->events[0], st) != hipSuccess) return SNAP_EHIP;
  for (int i = 0; i < ns; ++i)
    if (hipStreamWaitEvent(plan->streams[i], plan->events[0], 0) != hipSuccess) return SNAP_EHIP;
  for (size_t gi = 0; gi < plan->groups.size(); ++gi) {
    const int rc = launch_group(plan, a, plan->groups[gi], plan->streams[gi % ns]);
    if (rc != 0) return rc;
  }
  for (int i = 0; i < ns; ++i) {
    if (hipEventRecord(plan->events[1 + i], plan->streams[i]) != hipSuccess) return SNAP_EHIP;
    if (hipStreamWaitEvent(st, plan->events[1 + i], 0) != hipSuccess) return SNAP_EHIP;
  }
  return SNAP_SUCCESS;
}

// the pointers a captured graph has baked into its kernel arguments
static bool same_call(const KernelArgs& x, const KernelArgs& y) {
  return x.uhat == y.uhat && x.aux == y.aux && x.u == y.u && x.lam == y.lam &&
         x.stats == y.stats && x.grad_u == y.grad_u && x.grad_uhat == y.grad_uhat &&
         x.ws == y.ws && x.backward == y.backward;
}

// SNAP_FLAG_GRAPH: replay the call's launches from a graph captured on the
// first call with these arguments (the fork/join over the plan's streams is
// captured through its events).
static int run_graph(snap_plan plan, const KernelArgs& a, hipStream_t st) {
  if (st == nullptr) return run(plan, a, st);   // the null stream cannot be captured
  // one slab-row or spectral group is one kernel launch: a graph would only
  // add its replay
  if (plan->groups.size() == 1 && plan->groups[0].kind != 1) return run(plan, a, st);
  std::lock_guard<std::mutex> lock(plan->graph_mu);
  GraphSlot& g = plan->graphs[a.backward ? 1 : 0];
  if (!g.exec || !same_call(g.key, a)) {
    if (g.exec) {
      (void)hipGraphExecDestroy(g.exec);
      g.exec = nullptr;
    }
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return SNAP_EHIP;
    const int rc = run(plan, a, st);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(st, &graph);
    if (rc != 0 || ec != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc != 0 ? rc : SNAP_EHIP;
    }
    const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      g.exec = nullptr;
      return SNAP_EHIP;
    }
    g.key = a;
  }
  return hipGraphLaunch(g.exec, st) == hipSuccess ? SNAP_SUCCESS : SNAP_EHIP;
}

static int dispatch(snap_plan plan, const KernelArgs& a, hipStream_t st) {
  // the fork/join events and the timer are per plan: one call at a time
  std::lock_guard<std::mutex> lock(plan->run_mu);
  if (plan->opt.flags & SNAP_FLAG_GRAPH) return run_graph(plan, a, st);
  if (!plan->timer) return run(plan, a, st);
  tl_timer = plan->timer;
  const int rc = run(plan, a, st);
  tl_timer = nullptr;
  return rc;
}

int snap_project(snap_plan plan, const double* uhat, const double* aux, double* u_out,
                 double* lambda_out, snap_sample_stats* stats, void* workspace, void* stream) {
  if (!plan) return SNAP_EINVAL;
  if (plan->batch == 0) return SNAP_SUCCESS;
  if (!uhat || !u_out || !lambda_out || !stats || !workspace) return SNAP_EINVAL;
  if (plan->total_aux > 0 && !aux) return SNAP_EINVAL;
  if (u_out == uhat) return SNAP_EINVAL;
  if (((uintptr_t)workspace & 255) != 0) return SNAP_EINVAL;
  KernelArgs a{};
  a.descs = plan->d_descs;
  a.uhat = uhat;
  a.aux = aux;
  a.u = u_out;
  a.lam = lambda_out;
  a.stats = stats;
  a.ws = (unsigned char*)workspace;
  a.ws_off = plan->d_ws_off;
  a.opt = plan->opt;
  a.backward = 0;
  return dispatch(plan, a, (hipStream_t)stream);
}

int snap_project_noalloc(snap_plan plan, const double* uhat, const double* aux, double* u_out,
                         double* lambda_out, snap_sample_stats* stats, void* stream) {
  if (!plan) return SNAP_EINVAL;
  if (plan->batch == 0) return SNAP_SUCCESS;
  if (plan->ws_bytes > kStaticScratchBytes) return SNAP_EINVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != plan->device) return SNAP_EINVAL;
  void* ptr = scratch_ptr(dev);
  if (!ptr) return SNAP_EHIP;
  return snap_project(plan, uhat, aux, u_out, lambda_out, stats, ptr, stream);
}

int snap_project_backward(snap_plan plan, const double* u, const double* lambda, const double* aux,
                          void* workspace, const double* grad_u, double* grad_uhat,
                          snap_sample_stats* stats, void* stream) {
  if (!plan) return SNAP_EINVAL;
  if (plan->batch == 0) return SNAP_SUCCESS;
  if (!u || !lambda || !grad_u || !grad_uhat || !stats || !workspace) return SNAP_EINVAL;
  if (((uintptr_t)workspace & 255) != 0) return SNAP_EINVAL;
  KernelArgs a{};
  a.descs = plan->d_descs;
  a.uhat = nullptr;
  a.aux = aux;
  a.u = const_cast<double*>(u);
  a.lam = const_cast<double*>(lambda);
  a.stats = stats;
  a.grad_u = grad_u;
  a.grad_uhat = grad_uhat;
  a.ws = (unsigned char*)workspace;
  a.ws_off = plan->d_ws_off;
  a.opt = plan->opt;
  a.backward = 1;
  if (plan->total_aux > 0 && !aux) {
    // the slab kernels read aux (IC targets) unconditionally
    return SNAP_EINVAL;
  }
  return dispatch(plan, a, (hipStream_t)stream);
}

int snap_plan_describe(snap_plan plan, char* buf, size_t len, size_t* needed) {
  if (!plan || (len > 0 && !buf)) return SNAP_EINVAL;
  std::string t;
  for (size_t i = 0; i < plan->groups.size(); ++i) {
    const Group& g = plan->groups[i];
    char line[192];
    std::snprintf(line, sizeof(line), "group %zu: %s class %d, %d wavefronts per workgroup%s, %zu samples\n",
                  i, g.kind == 0 ? "slab" : (g.kind == 1 ? "band" : (g.kind == 2 ? "spectral" : "boundary-row")), g.cls,
                  g.kind == 0 ? slab_waves(g.cls) : (g.kind == 1 ? band_waves(g.cls) : 8),
                  g.kind == 1 && band_sides(g.cls) == 2 ? ", two-sided factorization" : "", g.ids.size());
    t += line;
  }
  if (needed) *needed = t.size();
  if (len > 0) {
    const size_t c = std::min(len - 1, t.size());
    std::memcpy(buf, t.data(), c);
    buf[c] = 0;
  }
  return SNAP_SUCCESS;
}

int snap_plan_group_classes(snap_plan plan, int32_t group, int32_t* classes, int32_t cap,
                            int32_t* count) {
  if (!plan || group < 0 || group >= (int32_t)plan->groups.size() || cap < 0 || (cap > 0 && !classes))
    return SNAP_EINVAL;
  const Group& g = plan->groups[group];
  std::vector<int> c = group_candidates(*plan, g);
  auto it = std::find(c.begin(), c.end(), g.cls);
  if (it != c.end()) std::rotate(c.begin(), it, it + 1);
  if (count) *count = (int32_t)c.size();
  for (int32_t i = 0; i < cap && i < (int32_t)c.size(); ++i) classes[i] = c[i];
  return SNAP_SUCCESS;
}

int snap_plan_set_group_class(snap_plan plan, int32_t group, int32_t cls) {
  if (!plan || group < 0 || group >= (int32_t)plan->groups.size()) return SNAP_EINVAL;
  int32_t c[16], n = 0;
  const int rc = snap_plan_group_classes(plan, group, c, 16, &n);
  if (rc != SNAP_SUCCESS) return rc;
  if (std::find(c, c + std::min<int32_t>(n, 16), cls) == c + std::min<int32_t>(n, 16)) return SNAP_EINVAL;
  std::lock_guard<std::mutex> lock(plan->graph_mu);
  plan->groups[group].cls = cls;
  for (auto& gr : plan->graphs)
    if (gr.exec) {
      (void)hipGraphExecDestroy(gr.exec);
      gr.exec = nullptr;
    }
  return SNAP_SUCCESS;
}

int snap_plan_set_kernel_timing(snap_plan plan, int32_t enable) {
  if (!plan) return SNAP_EINVAL;
  if (plan->opt.flags & SNAP_FLAG_GRAPH) return SNAP_EUNSUPPORTED;
  if (!enable) { free_timer(plan); return SNAP_SUCCESS; }
  if (plan->timer) { plan->timer->marks.clear(); plan->timer->dropped = 0; return SNAP_SUCCESS; }
  KernelTimer* t = new (std::nothrow) KernelTimer();
  if (!t) return SNAP_ENOMEM;
  t->pool.assign(kTimerEvents, nullptr);
  for (auto& e : t->pool)
    if (hipEventCreate(&e) != hipSuccess) {
      for (auto& f : t->pool)
        if (f) (void)hipEventDestroy(f);
      delete t;
      return SNAP_EHIP;
    }
  t->marks.reserve(kTimerEvents);
  plan->timer = t;
  return SNAP_SUCCESS;
}

int snap_plan_kernel_times(snap_plan plan, int32_t kernel, double* total_ms, int64_t* launches,
                           int64_t* dropped) {
  if (!plan || !plan->timer || kernel < 0 || kernel >= kTimedCount) return SNAP_EINVAL;
  KernelTimer* t = plan->timer;
  double ms = 0.0;
  int64_t n = 0;
  // marks come in (begin, end) pairs per launch and kernel
  std::vector<int> open(kTimedCount, -1);
  for (const auto& mk : t->marks) {
    if (mk.first != kernel) continue;
    if (open[kernel] < 0) { open[kernel] = mk.second; continue; }
    if (hipEventSynchronize(t->pool[mk.second]) != hipSuccess) return SNAP_EHIP;
    float e = 0.0f;
    if (hipEventElapsedTime(&e, t->pool[open[kernel]], t->pool[mk.second]) != hipSuccess) return SNAP_EHIP;
    ms += e;
    ++n;
    open[kernel] = -1;
  }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = n;
  if (dropped) *dropped = t->dropped;
  return SNAP_SUCCESS;
}

int snap_plan_reset_kernel_times(snap_plan plan) {
  if (!plan || !plan->timer) return SNAP_EINVAL;
  for (const auto& mk : plan->timer->marks)
    if (hipEventSynchronize(plan->timer->pool[mk.second]) != hipSuccess) return SNAP_EHIP;
  plan->timer->marks.clear();
  plan->timer->dropped = 0;
  return SNAP_SUCCESS;
}

int snap_plan_destroy(snap_plan plan) {
  if (!plan) return SNAP_EINVAL;
  free_plan(plan);
  return SNAP_SUCCESS;
}

const char* snap_error_string(int code) {
  switch (code) {
    case SNAP_SUCCESS: return "success";
    case SNAP_EINVAL: return "invalid argument";
    case SNAP_EHIP: return "HIP runtime error";
    case SNAP_ENOMEM: return "out of memory";
    case SNAP_EUNSUPPORTED: return "unsupported family or size";
    default: return "unknown error";
  }
}

const char* snap_status_string(int status) {
  switch (status) {
    case SNAP_ST_CONVERGED: return "converged";
    case SNAP_ST_MAX_ITER: return "max_iter";
    case SNAP_ST_LS_FAIL: return "line_search_failed";
    case SNAP_ST_NONFINITE: return "nonfinite";
    case SNAP_ST_SINGULAR_PIVOT: return "singular_pivot";
    case SNAP_ST_HESSIAN_FLOOR: return "hessian_floor";
    default: return "unknown";
  }
}

}  // extern "C"
