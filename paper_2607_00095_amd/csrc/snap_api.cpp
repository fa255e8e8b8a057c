// Host side of the C ABI declared in include/snap.h: plan construction
// (shapes, groupings, workspace layout; the sparsity structure is fixed once,
// as the paper exploits for repeated factorizations, Sec. III-B/III-C), and
// stream-ordered launches of the family kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "snap.h"
#include "snap_device.hpp"

namespace snap {
int slab_class(int nx, int nt);
int slab_launch(const KernelArgs& a, int cls, bool mixed, hipStream_t st);
int band_class(int nx, int nt);
int band_launch(const KernelArgs& a, int cls, bool mixed, hipStream_t st);
size_t band_workspace_bytes(int nx, int nt, bool mixed);
}  // namespace snap

using namespace snap;

namespace {

// Samples sharing one kernel instantiation (shapes may differ: every kernel
// reads its sample's shape from the descriptor).  `kind` 0 = slab rows,
// 1 = banded; `cls` = instantiation index; ids sorted by decreasing cost so
// the longest samples start first.
struct Group {
  int kind, cls;
  double cost = 0.0;
  std::vector<int32_t> ids;
  int32_t* d_ids = nullptr;
};

constexpr int kStreams = 4;   // groups are spread over this many internal streams

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
  size_t ws_bytes = 0;
  int64_t total_vars = 0, total_rows = 0, total_aux = 0;
  int device = 0;
  std::vector<hipStream_t> streams;     // fork/join of independent groups
  std::vector<hipEvent_t> events;       // [0] fork, [1..] join per stream
  GraphSlot graphs[2];                  // SNAP_FLAG_GRAPH: forward, backward
  std::mutex graph_mu;
};

namespace {

int64_t rows_of(const snap_sample_desc& d) {
  switch (d.family) {
    case SNAP_MASS_IC:
    case SNAP_FISHER_KPP: return (int64_t)d.nx + d.nt - 1;
    case SNAP_BURGERS_LF: return (int64_t)d.nx * (d.nt - 1);
    default: return -1;
  }
}

int64_t aux_of(const snap_sample_desc& d) {
  switch (d.family) {
    case SNAP_MASS_IC: return d.nx + 1;
    case SNAP_FISHER_KPP: return d.nx;
    default: return 0;
  }
}

void free_plan(snap_plan p) {
  if (!p) return;
  for (auto& g : p->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  for (auto& e : p->events) (void)hipEventDestroy(e);
  for (auto& s : p->streams) (void)hipStreamDestroy(s);
  for (auto& g : p->groups)
    if (g.d_ids) (void)hipFree(g.d_ids);
  if (p->d_descs) (void)hipFree(p->d_descs);
  if (p->d_ws_off) (void)hipFree(p->d_ws_off);
  delete p;
}

bool options_valid(const snap_options& o) {
  return o.tol_h > 0 && o.tol_s > 0 && o.max_newton >= 1 && o.max_ls >= 0 &&
         (o.precision == SNAP_PREC_FP64 || o.precision == SNAP_PREC_MIXED);
}

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
    if (d.nx < 1 || d.nt < 1 || d.ny != 1 || d.var_off < 0 || d.row_off < 0 || d.aux_off < 0) {
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
    } else if (d.family == SNAP_BURGERS_LF) {
      kind = 1;
      cls = (d.dt > 0.0 && d.dx > 0.0) ? band_class(d.nx, d.nt) : -1;
      if (cls > 0) need = band_workspace_bytes(d.nx, d.nt, mixed);
      // factorization work ~ rows x (block bandwidth)^2
      cost[s] = (double)d.nx * (d.nt - 1) * (double)(cls + 1) * (cls + 1) * 256.0;
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

static int launch_group(const snap_plan plan, KernelArgs a, const Group& g, hipStream_t st) {
  const bool mixed = plan->opt.precision == SNAP_PREC_MIXED;
  a.order = g.d_ids;
  a.count = (int32_t)g.ids.size();
  return g.kind == 0 ? slab_launch(a, g.cls, mixed, st) : band_launch(a, g.cls, mixed, st);
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
  return (plan->opt.flags & SNAP_FLAG_GRAPH) ? run_graph(plan, a, st) : run(plan, a, st);
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
    default: return "unknown";
  }
}

}  // extern "C"
