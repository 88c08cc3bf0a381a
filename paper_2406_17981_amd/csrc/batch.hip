// Multi-problem batches and the autotuner.
//
// sfft_apply_multi runs independent products (uneven grids, block sizes,
// right-hand-side counts) as one HIP graph, replayed with a single graph
// launch. Two forms are captured: per-problem chains (each problem's launches
// on its own forked stream, so problems run side by side) and grouped lanes
// (problems of equal level lengths form a lane on its own forked stream; step
// k of every member in stage k, the entries of one kernel in one launch over
// a table). The first call with an argument set times both and keeps the
// faster (SFFT_BATCH_MODE=chains|grouped forces one). Instantiated graphs are
// cached per argument set (plans, vectors, workspace); a plan's graphs are
// dropped when the plan is destroyed.
//
// sfft_plan_autotune times the candidate schedules (breadth-first / depth-
// first) and leaf right-hand-side groupings of a plan on the device and keeps
// the fastest; results persist in a JSON-lines cache file (SFFT_TUNE_CACHE,
// default $HOME/.cache/sfft_autotune.jsonl) keyed by device architecture,
// method, dtype, block size, grid, symbol storage and right-hand sides.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "plan_internal.hpp"

namespace {

constexpr int kSideStreams = 4;
constexpr size_t kMaxGraphs = 32;

struct GraphEntry {
  std::vector<uintptr_t> key;
  std::vector<const sfft_plan_s*> plans;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* table = nullptr;  // device copy of the grouped launches' entries
  int form = 0;           // 0 per-problem chains, 1 grouped stages
  uint64_t last_use = 0;
};

std::mutex g_mu;
std::vector<GraphEntry> g_graphs;
uint64_t g_tick = 0;
hipStream_t g_cap = nullptr;
hipStream_t g_side[kSideStreams] = {nullptr};
int g_dev = -1;

void destroy_entry(GraphEntry& e) {
  if (e.exec) (void)hipGraphExecDestroy(e.exec);
  if (e.graph) (void)hipGraphDestroy(e.graph);
  if (e.table) (void)hipFree(e.table);
  e.exec = nullptr;
  e.graph = nullptr;
  e.table = nullptr;
}

sfft_status ensure_streams() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return sfft_rt_hip_fail(e, "hipGetDevice");
  if (g_dev == dev && g_cap) return SFFT_OK;
  if (g_cap) {
    (void)hipStreamDestroy(g_cap);
    for (auto& s : g_side) (void)hipStreamDestroy(s);
  }
  e = hipStreamCreateWithFlags(&g_cap, hipStreamNonBlocking);
  if (e != hipSuccess) return sfft_rt_hip_fail(e, "capture stream");
  for (auto& s : g_side) {
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return sfft_rt_hip_fail(e, "side stream");
  }
  g_dev = dev;
  return SFFT_OK;
}

bool graphs_enabled() {
  const char* v = std::getenv("SFFT_NO_GRAPH");
  return !(v && v[0] && v[0] != '0');
}

// Requested batch graph form: -1 timed choice (default), 0 chains, 1 grouped.
int batch_form_request() {
  const char* v = std::getenv("SFFT_BATCH_MODE");
  if (v && std::strcmp(v, "chains") == 0) return 0;
  if (v && std::strcmp(v, "grouped") == 0) return 1;
  return -1;
}

int g_last_form = -1;  // form of the graph launched by the last graph call

// Captures the batch on g_cap with one forked stream per problem (problems
// beyond the side streams share them in turn), each problem's launches in its
// own schedule.
sfft_status capture_chains(int nprob, const sfft_plan* plans, const void* const* x, void* const* y,
                           const int64_t* nrhs, char* ws, const std::vector<size_t>& off,
                           const std::vector<size_t>& wsz, hipGraph_t* out) {
  std::vector<unsigned> masks(nprob);
  for (int i = 0; i < nprob; ++i) {  // profiling event pairs are not captured
    masks[i] = plans[i]->prof_mask;
    plans[i]->prof_mask = 0;
  }
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> done(nprob, nullptr);
  sfft_status s = SFFT_OK;
  hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  for (int i = 0; i < nprob && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&done[i], hipEventDisableTiming);
  if (e != hipSuccess) s = sfft_rt_hip_fail(e, "batch events");
  bool capturing = false;
  if (s == SFFT_OK) {
    e = hipStreamBeginCapture(g_cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) s = sfft_rt_hip_fail(e, "begin capture");
    else capturing = true;
  }
  if (s == SFFT_OK) {
    e = hipEventRecord(fork, g_cap);
    if (e != hipSuccess) s = sfft_rt_hip_fail(e, "fork");
  }
  for (int i = 0; i < nprob && s == SFFT_OK; ++i) {
    hipStream_t si = g_side[i % kSideStreams];
    e = hipStreamWaitEvent(si, fork, 0);
    if (e != hipSuccess) {
      s = sfft_rt_hip_fail(e, "fork wait");
      break;
    }
    s = sfft_rt_apply_one(plans[i], x[i], y[i], nrhs[i], wsz[i] ? ws + off[i] : nullptr, wsz[i], si);
    if (s != SFFT_OK) break;
    e = hipEventRecord(done[i], si);
    if (e != hipSuccess) s = sfft_rt_hip_fail(e, "join record");
  }
  for (int i = 0; i < nprob && s == SFFT_OK; ++i) {
    e = hipStreamWaitEvent(g_cap, done[i], 0);
    if (e != hipSuccess) s = sfft_rt_hip_fail(e, "join wait");
  }
  if (capturing) {
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(g_cap, &g);
    if (s == SFFT_OK && e != hipSuccess) s = sfft_rt_hip_fail(e, "end capture");
    if (s == SFFT_OK) *out = g;
    else if (g) (void)hipGraphDestroy(g);
  }
  if (fork) (void)hipEventDestroy(fork);
  for (auto ev : done)
    if (ev) (void)hipEventDestroy(ev);
  for (int i = 0; i < nprob; ++i) plans[i]->prof_mask = masks[i];
  return s;
}

// One launch of a batch stage: the same pass (or leaf) of several problems
// over a table of entries, or one problem's launch of its own where the
// length has no grouped kernel.
struct GroupLaunch {
  int kind = 0;  // 0 grouped pass, 1 grouped leaf, 2 single pass, 3 single leaf
  const sfft::AxisOps* ops = nullptr;
  int mode = 0, half = 0;
  sfft::leaf_group_fn lgroup = nullptr;
  sfft::pass_fn single = nullptr;
  int rb = 1;
  size_t smem = 0;
  int64_t blocks = 0;
  size_t first = 0, count = 0;  // entries in the flat table
};

// The member problems of a lane as stages of the breadth-first schedule,
// step k of every member in stage k (a d-level problem has 2d - 1 steps:
// forward passes of levels 1..d-1, the leaf, inverse passes of levels
// d-1..1); inside a stage the entries of one kernel form one grouped launch.
sfft_status build_stages(const std::vector<int>& members, const sfft_plan* plans, const void* const* x,
                         void* const* y, const int64_t* nrhs, char* ws, const std::vector<size_t>& off,
                         std::vector<std::vector<GroupLaunch>>& stages, std::vector<sfft::PassArgs>& table) {
  struct Item {
    int kind;  // 0 pass, 1 leaf
    sfft::PassArgs a;
    const sfft::AxisOps* ops;
    int mode;
    LeafSel sel;
  };
  std::vector<std::vector<Item>> items;
  for (int i : members) {
    const sfft_plan_s* p = plans[i];
    const int d = p->d;
    const int64_t nv = nrhs[i] * p->b;
    const int64_t V = nv * p->s;
    const size_t vb = (size_t)V * p->esz;
    std::vector<char*> blk(d > 1 ? d - 1 : 1);
    size_t o = 0;
    for (int l = 0; l + 1 < d; ++l) {
      blk[l] = ws + off[i] + o;
      o += (size_t)(int64_t(2) << l) * vb;
    }
    std::vector<Item> seq;
    for (int l = 0; l + 1 < d; ++l) {
      Item it{0, sfft_rt_pass_args(p, l, nv), p->ops[l], 0, {}};
      it.a.in = l == 0 ? x[i] : (const void*)blk[l - 1];
      it.a.in_bs = V;
      it.a.nq = int64_t(1) << l;
      it.a.out = blk[l];
      it.a.out1 = blk[l] + vb;
      it.a.out_bs = 2 * V;
      it.a.use_phase = 1;
      seq.push_back(it);
    }
    {
      Item it{1, {}, p->ops[d - 1], 0, {}};
      const void* in = d == 1 ? x[i] : (const void*)blk[d - 2];
      void* out = d == 1 ? y[i] : (void*)blk[d - 2];
      sfft_status s = sfft_rt_leaf_args(p, in, out, V, int64_t(1) << (d - 1), nrhs[i], &it.a, &it.sel);
      if (s != SFFT_OK) return s;
      seq.push_back(it);
    }
    for (int l = d - 2; l >= 0; --l) {
      Item it{0, sfft_rt_pass_args(p, l, nv), p->ops[l], 1, {}};
      it.a.in = blk[l];
      it.a.in1 = blk[l] + vb;
      it.a.in_bs = 2 * V;
      it.a.nq = int64_t(1) << l;
      it.a.out = l == 0 ? y[i] : (void*)blk[l - 1];
      it.a.out_bs = V;
      it.a.use_phase = 1;
      seq.push_back(it);
    }
    if (items.size() < seq.size()) items.resize(seq.size());
    for (size_t k = 0; k < seq.size(); ++k) items[k].push_back(seq[k]);
  }
  stages.assign(items.size(), {});
  for (size_t k = 0; k < items.size(); ++k) {
    std::vector<bool> used(items[k].size(), false);
    for (size_t u = 0; u < items[k].size(); ++u) {
      if (used[u]) continue;
      const Item& head = items[k][u];
      GroupLaunch g;
      std::vector<sfft::PassArgs> ents;
      if (head.kind == 0) {
        g.ops = head.ops;
        g.mode = head.mode;
        if (!head.ops->strided_group[head.mode][0]) {  // no grouped kernel: a launch of its own
          g.kind = 2;
          g.single = head.ops->strided[head.mode];
          ents.push_back(head.a);
          used[u] = true;
        } else {
          g.kind = 0;
          for (size_t v = u; v < items[k].size(); ++v)
            if (!used[v] && items[k][v].kind == 0 && items[k][v].ops == head.ops && items[k][v].mode == head.mode) {
              ents.push_back(items[k][v].a);
              used[v] = true;
            }
          // few workgroups in all: half-size ones, as for a launch of its own
          int64_t total = 0;
          for (auto a : ents) {
            const int64_t nb = head.ops->strided_prep[0](a);
            if (nb < 0) return sfft_rt_fail(SFFT_UNSUPPORTED, "batched pass beyond the 1-D grid");
            total += nb;
          }
          g.half = (head.ops->strided_prep[1] && total < sfft::kHalfTilesBelow) ? 1 : 0;
          g.blocks = 0;
          for (auto& a : ents) {
            const int64_t nb = head.ops->strided_prep[g.half](a);
            if (nb < 0) return sfft_rt_fail(SFFT_UNSUPPORTED, "batched pass beyond the 1-D grid");
            a.blk_begin = (uint32_t)g.blocks;
            g.blocks += nb;
          }
        }
      } else {
        sfft::PassArgs a0 = head.a;
        size_t smem0 = 0;
        if (!head.sel.prep || !head.sel.group || head.sel.prep(a0, &smem0) <= 0) {
          g.kind = 3;
          g.single = head.sel.single;
          ents.push_back(head.a);
          used[u] = true;
        } else {
          g.kind = 1;
          g.lgroup = head.sel.group;
          g.rb = a0.rb;
          g.smem = smem0;
          for (size_t v = u; v < items[k].size(); ++v) {
            const Item& it = items[k][v];
            if (used[v] || it.kind != 1 || it.sel.group != head.sel.group) continue;
            sfft::PassArgs a = it.a;
            size_t smem = 0;
            const int64_t nb = it.sel.prep(a, &smem);
            if (nb <= 0 || a.rb != g.rb || smem != g.smem) continue;
            a.blk_begin = (uint32_t)g.blocks;
            g.blocks += nb;
            ents.push_back(a);
            used[v] = true;
          }
        }
      }
      if (g.blocks >= sfft::kIdx32) return sfft_rt_fail(SFFT_UNSUPPORTED, "batched launch beyond the 1-D grid");
      g.first = table.size();
      g.count = ents.size();
      table.insert(table.end(), ents.begin(), ents.end());
      stages[k].push_back(g);
    }
  }
  return SFFT_OK;
}

// Lanes of the grouped form: split problems with the same level lengths (so
// the same pass kernels at every step) share a lane; embedding problems and
// problems without right-hand sides have none.
std::vector<std::vector<int>> make_lanes(int nprob, const sfft_plan* plans, const int64_t* nrhs) {
  std::vector<std::vector<int>> lanes;
  for (int i = 0; i < nprob; ++i) {
    const sfft_plan_s* p = plans[i];
    if (p->method != SFFT_SPLIT || nrhs[i] == 0) continue;
    bool placed = false;
    for (auto& ln : lanes) {
      const sfft_plan_s* h = plans[ln[0]];
      bool same = h->d == p->d && h->dtype == p->dtype;
      for (int l = 0; same && l < p->d; ++l) same = h->n[l] == p->n[l];
      if (same) {
        ln.push_back(i);
        placed = true;
        break;
      }
    }
    if (!placed) lanes.push_back({i});
  }
  return lanes;
}

// Captures the batch on g_cap as grouped lanes: every lane (and every
// embedding problem) on a forked side stream, a lane's stages in order on its
// stream with one launch per kernel per stage, all joined back at the end.
// The grouped launches read their entries from dtab (uploaded before the
// capture).
sfft_status capture_grouped(int nprob, const sfft_plan* plans, const void* const* x, void* const* y,
                            const int64_t* nrhs, char* ws, const std::vector<size_t>& off,
                            const std::vector<size_t>& wsz, hipGraph_t* out, void** dtab_out) {
  const std::vector<std::vector<int>> lanes = make_lanes(nprob, plans, nrhs);
  std::vector<std::vector<std::vector<GroupLaunch>>> lane_stages(lanes.size());
  std::vector<sfft::PassArgs> table;
  sfft_status s = SFFT_OK;
  for (size_t j = 0; j < lanes.size() && s == SFFT_OK; ++j)
    s = build_stages(lanes[j], plans, x, y, nrhs, ws, off, lane_stages[j], table);
  if (s != SFFT_OK) return s;
  sfft::PassArgs* dtab = nullptr;
  if (!table.empty()) {
    hipError_t e = hipMalloc(&dtab, table.size() * sizeof(sfft::PassArgs));
    if (e == hipSuccess) e = hipMemcpy(dtab, table.data(), table.size() * sizeof(sfft::PassArgs), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      if (dtab) (void)hipFree(dtab);
      return sfft_rt_hip_fail(e, "batch table");
    }
  }
  std::vector<int> embeds;
  for (int i = 0; i < nprob; ++i)
    if (plans[i]->method != SFFT_SPLIT) embeds.push_back(i);
  const size_t nchain = lanes.size() + embeds.size();
  std::vector<unsigned> masks(nprob);
  for (int i = 0; i < nprob; ++i) {  // profiling event pairs are not captured
    masks[i] = plans[i]->prof_mask;
    plans[i]->prof_mask = 0;
  }
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> done(nchain, nullptr);
  hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  for (size_t c = 0; c < nchain && e == hipSuccess; ++c) e = hipEventCreateWithFlags(&done[c], hipEventDisableTiming);
  if (e != hipSuccess) s = sfft_rt_hip_fail(e, "batch events");
  bool capturing = false;
  if (s == SFFT_OK) {
    e = hipStreamBeginCapture(g_cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) s = sfft_rt_hip_fail(e, "begin capture");
    else capturing = true;
  }
  if (s == SFFT_OK) {
    e = hipEventRecord(fork, g_cap);
    if (e != hipSuccess) s = sfft_rt_hip_fail(e, "fork");
  }
  for (size_t c = 0; c < nchain && s == SFFT_OK; ++c) {
    hipStream_t si = g_side[c % kSideStreams];
    e = hipStreamWaitEvent(si, fork, 0);
    if (e != hipSuccess) {
      s = sfft_rt_hip_fail(e, "fork wait");
      break;
    }
    if (c < lanes.size()) {
      for (const auto& stage : lane_stages[c]) {
        for (const GroupLaunch& g : stage) {
          switch (g.kind) {
            case 0: e = g.ops->strided_group[g.mode][g.half](dtab + g.first, (int)g.count, g.blocks, si); break;
            case 1: e = g.lgroup(dtab + g.first, (int)g.count, g.blocks, g.rb, g.smem, si); break;
            default: e = g.single(table[g.first], si); break;
          }
          if (e != hipSuccess) break;
        }
        if (e != hipSuccess) break;
      }
      if (e != hipSuccess) {
        s = sfft_rt_hip_fail(e, "batch launch");
        break;
      }
    } else {  // embedding baseline: its own chain
      const int i = embeds[c - lanes.size()];
      s = sfft_rt_apply_one(plans[i], x[i], y[i], nrhs[i], wsz[i] ? ws + off[i] : nullptr, wsz[i], si);
      if (s != SFFT_OK) break;
    }
    e = hipEventRecord(done[c], si);
    if (e != hipSuccess) s = sfft_rt_hip_fail(e, "join record");
  }
  for (size_t c = 0; c < nchain && s == SFFT_OK; ++c) {
    e = hipStreamWaitEvent(g_cap, done[c], 0);
    if (e != hipSuccess) s = sfft_rt_hip_fail(e, "join wait");
  }
  if (capturing) {
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(g_cap, &g);
    if (s == SFFT_OK && e != hipSuccess) s = sfft_rt_hip_fail(e, "end capture");
    if (s == SFFT_OK) *out = g;
    else if (g) (void)hipGraphDestroy(g);
  }
  if (fork) (void)hipEventDestroy(fork);
  for (auto ev : done)
    if (ev) (void)hipEventDestroy(ev);
  for (int i = 0; i < nprob; ++i) plans[i]->prof_mask = masks[i];
  if (s == SFFT_OK) *dtab_out = dtab;
  else if (dtab) (void)hipFree(dtab);
  return s;
}

std::string tune_cache_path() {
  const char* p = std::getenv("SFFT_TUNE_CACHE");
  if (p && p[0]) return p;
  const char* h = std::getenv("HOME");
  return std::string(h ? h : ".") + "/.cache/sfft_autotune.jsonl";
}

std::string tune_key(const sfft_plan_s* p, int64_t nrhs) {
  hipDeviceProp_t prop;
  int dev = 0;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  std::ostringstream k;
  k << arch << "|" << (p->method == SFFT_SPLIT ? "split" : "embed") << "|" << (p->dtype == SFFT_C64 ? "c64" : "c128")
    << "|b" << p->b << "|";
  for (int l = 0; l < p->d; ++l) k << (l ? "x" : "") << p->n[l];
  k << "|nrhs" << nrhs << "|mirror" << p->compressed;
  return k.str();
}

// tiles: one digit per level (the plan's tile_mode), "" when not recorded
bool tune_lookup(const std::string& key, int* sched, int* rb, std::string* tiles) {
  std::ifstream f(tune_cache_path());
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {  // later lines win
    const std::string tag = "\"key\": \"" + key + "\"";
    if (line.find(tag) == std::string::npos) continue;
    int s = 0, r = 0;
    const size_t ps = line.find("\"sched\": "), pr = line.find("\"rb\": ");
    if (ps == std::string::npos || pr == std::string::npos) continue;
    s = std::atoi(line.c_str() + ps + 9);
    r = std::atoi(line.c_str() + pr + 6);
    if (s >= SFFT_SCHED_BREADTH && s <= SFFT_SCHED_SLAB && r >= 0) {
      *sched = s;
      *rb = r;
      tiles->clear();
      const size_t pt = line.find("\"tiles\": \"");
      if (pt != std::string::npos)
        for (size_t i = pt + 10; i < line.size() && line[i] >= '0' && line[i] <= '2'; ++i) tiles->push_back(line[i]);
      found = true;
    }
  }
  return found;
}

void tune_store(const std::string& key, int sched, int rb, const std::string& tiles, double us) {
  std::ofstream f(tune_cache_path(), std::ios::app);
  if (!f) return;  // a read-only home leaves tuning per process
  f << "{\"key\": \"" << key << "\", \"sched\": " << sched << ", \"rb\": " << rb << ", \"tiles\": \"" << tiles
    << "\", \"us\": " << us << "}\n";
}

}  // namespace

void sfft_rt_forget_plan(const sfft_plan_s* p) {
  std::lock_guard<std::mutex> g(g_mu);
  for (size_t i = 0; i < g_graphs.size();) {
    bool uses = false;
    for (auto q : g_graphs[i].plans) uses |= (q == p);
    if (uses) {
      destroy_entry(g_graphs[i]);
      g_graphs.erase(g_graphs.begin() + i);
    } else {
      ++i;
    }
  }
}

namespace {

#define HIP_OK(expr, what)                                \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return sfft_rt_hip_fail(e_, what); \
  } while (0)

// Fork / join events of sfft_apply_each on the current device's side
// streams (created once with them, reused under g_mu).
hipEvent_t g_fork = nullptr;
hipEvent_t g_join[kSideStreams] = {nullptr};
int g_ev_dev = -1;

sfft_status ensure_events() {
  if (g_ev_dev == g_dev && g_fork) return SFFT_OK;
  if (g_fork) {
    (void)hipEventDestroy(g_fork);
    for (auto& e : g_join) (void)hipEventDestroy(e);
  }
  hipError_t e = hipEventCreateWithFlags(&g_fork, hipEventDisableTiming);
  for (int i = 0; i < kSideStreams && e == hipSuccess; ++i)
    e = hipEventCreateWithFlags(&g_join[i], hipEventDisableTiming);
  if (e != hipSuccess) return sfft_rt_hip_fail(e, "batch events");
  g_ev_dev = g_dev;
  return SFFT_OK;
}

}  // namespace

extern "C" {

sfft_status sfft_apply_each(int nprob, const sfft_plan* plans, const void* const* x, void* const* y,
                            const int64_t* nrhs, void* const* workspaces, const size_t* ws_bytes, void* stream,
                            sfft_status* status) {
  if (nprob < 0 || (nprob > 0 && (!plans || !x || !y || !nrhs || !workspaces || !ws_bytes || !status)))
    return sfft_rt_fail(SFFT_INVALID_ARG, "null argument");
  if (nprob == 0) return SFFT_OK;
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(g_mu);
  sfft_status s = ensure_streams();
  if (s == SFFT_OK) s = ensure_events();
  if (s != SFFT_OK) return s;
  HIP_OK(hipEventRecord(g_fork, st), "fork record");
  const int nside = nprob < kSideStreams ? nprob : kSideStreams;
  for (int k = 0; k < nside; ++k) HIP_OK(hipStreamWaitEvent(g_side[k], g_fork, 0), "fork wait");
  for (int i = 0; i < nprob; ++i) {
    status[i] = plans[i] ? sfft_rt_apply_one(plans[i], x[i], y[i], nrhs[i], workspaces[i], ws_bytes[i],
                                             g_side[i % kSideStreams])
                         : sfft_rt_fail(SFFT_INVALID_ARG, "plan is null");
  }
  for (int k = 0; k < nside; ++k) {
    HIP_OK(hipEventRecord(g_join[k], g_side[k]), "join record");
    HIP_OK(hipStreamWaitEvent(st, g_join[k], 0), "join wait");
  }
  return SFFT_OK;
}

sfft_status sfft_apply_multi(int nprob, const sfft_plan* plans, const void* const* x, void* const* y,
                             const int64_t* nrhs, void* workspace, size_t ws_bytes, void* stream) {
  if (nprob < 0 || (nprob > 0 && (!plans || !x || !y || !nrhs))) return sfft_rt_fail(SFFT_INVALID_ARG, "null argument");
  size_t need = 0;
  sfft_status s = sfft_workspace_size_multi(nprob, plans, nrhs, &need);
  if (s != SFFT_OK) return s;
  if (need > 0 && (!workspace || ws_bytes < need)) return sfft_rt_fail(SFFT_INVALID_ARG, "workspace too small");
  std::vector<size_t> off(nprob), wsz(nprob);
  size_t o = 0;
  for (int i = 0; i < nprob; ++i) {
    wsz[i] = nrhs[i] > 0 ? sfft_rt_align256(sfft_rt_breadth_workspace_elems(plans[i], nrhs[i]) * plans[i]->esz) : 0;
    off[i] = o;
    o += wsz[i];
  }
  hipStream_t st = (hipStream_t)stream;
  if (nprob <= 1 || !graphs_enabled()) {
    for (int i = 0; i < nprob; ++i) {
      s = sfft_rt_apply_one(plans[i], x[i], y[i], nrhs[i], wsz[i] ? (char*)workspace + off[i] : nullptr, wsz[i], st);
      if (s != SFFT_OK) return s;
    }
    return SFFT_OK;
  }
  std::vector<uintptr_t> key;
  key.push_back((uintptr_t)nprob);
  key.push_back((uintptr_t)workspace);
  for (int i = 0; i < nprob; ++i) {
    key.push_back((uintptr_t)plans[i]);
    key.push_back((uintptr_t)x[i]);
    key.push_back((uintptr_t)y[i]);
    key.push_back((uintptr_t)nrhs[i]);
    key.push_back((uintptr_t)plans[i]->sched);
    key.push_back((uintptr_t)plans[i]->rb_pref);
    uintptr_t tm = 0;
    for (int l = 0; l < kMaxD; ++l) tm = tm * 3 + (uintptr_t)plans[i]->tile_mode[l];
    key.push_back(tm);
  }
  const int req = batch_form_request();
  key.push_back((uintptr_t)(req + 1));
  std::lock_guard<std::mutex> g(g_mu);
  if ((s = ensure_streams()) != SFFT_OK) return s;
  for (auto& e : g_graphs) {
    if (e.key == key) {
      e.last_use = ++g_tick;
      hipError_t he = hipGraphLaunch(e.exec, st);
      if (he != hipSuccess) return sfft_rt_hip_fail(he, "graph launch");
      g_last_form = e.form;
      return SFFT_OK;
    }
  }
  // argument checks happen outside capture so an invalid call never starts one
  for (int i = 0; i < nprob; ++i) {
    if (!plans[i] || nrhs[i] < 0 || (nrhs[i] > 0 && (!x[i] || !y[i] || x[i] == y[i])))
      return sfft_rt_fail(SFFT_INVALID_ARG, "bad problem entry");
  }
  // capture and instantiate the requested form(s)
  GraphEntry cand[2];
  bool have[2] = {false, false};
  for (int f = 0; f < 2; ++f) {
    if (req >= 0 && f != req) continue;
    GraphEntry& ent = cand[f];
    ent.key = key;
    ent.form = f;
    for (int i = 0; i < nprob; ++i) ent.plans.push_back(plans[i]);
    s = f == 0 ? capture_chains(nprob, plans, x, y, nrhs, (char*)workspace, off, wsz, &ent.graph)
               : capture_grouped(nprob, plans, x, y, nrhs, (char*)workspace, off, wsz, &ent.graph, &ent.table);
    hipError_t he = hipSuccess;
    if (s == SFFT_OK) {
      he = hipGraphInstantiate(&ent.exec, ent.graph, nullptr, nullptr, 0);
      if (he != hipSuccess) s = sfft_rt_hip_fail(he, "graph instantiate");
    }
    if (s != SFFT_OK) {
      destroy_entry(ent);
      // a timed choice keeps going with the form that did capture
      if (req >= 0 || (f == 1 && !have[0])) {
        for (auto& c : cand) destroy_entry(c);
        return s;
      }
      continue;
    }
    have[f] = true;
  }
  int pick = have[0] ? 0 : 1;
  if (have[0] && have[1]) {
    // both replay the same launches' results (bit for bit); time them on the
    // caller's stream after its pending work: one warm-up replay each, then
    // three trials of `reps` replays (about 2 ms a trial), fastest trial wins
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    double best[2] = {1e300, 1e300};
    for (int f = 0; f < 2 && he == hipSuccess; ++f) {
      float ms = 0.f;
      he = hipEventRecord(e0, st);
      if (he == hipSuccess) he = hipGraphLaunch(cand[f].exec, st);
      if (he == hipSuccess) he = hipEventRecord(e1, st);
      if (he == hipSuccess) he = hipEventSynchronize(e1);
      if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
      const int reps = ms > 0.f ? (int)std::min(20.0, std::max(2.0, 2.0 / ms)) : 20;
      for (int trial = 0; trial < 3 && he == hipSuccess; ++trial) {
        he = hipEventRecord(e0, st);
        for (int r = 0; r < reps && he == hipSuccess; ++r) he = hipGraphLaunch(cand[f].exec, st);
        if (he == hipSuccess) he = hipEventRecord(e1, st);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (he == hipSuccess) best[f] = std::min(best[f], (double)ms / reps);
      }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (he != hipSuccess) {
      for (auto& c : cand) destroy_entry(c);
      return sfft_rt_hip_fail(he, "batch form timing");
    }
    pick = best[1] < best[0] ? 1 : 0;
    destroy_entry(cand[1 - pick]);
  }
  if (g_graphs.size() >= kMaxGraphs) {  // evict the least recently used
    size_t victim = 0;
    for (size_t i = 1; i < g_graphs.size(); ++i)
      if (g_graphs[i].last_use < g_graphs[victim].last_use) victim = i;
    destroy_entry(g_graphs[victim]);
    g_graphs.erase(g_graphs.begin() + victim);
  }
  cand[pick].last_use = ++g_tick;
  g_graphs.push_back(cand[pick]);
  hipError_t he = hipGraphLaunch(g_graphs.back().exec, st);
  if (he != hipSuccess) return sfft_rt_hip_fail(he, "graph launch");
  g_last_form = pick;
  return SFFT_OK;
}

int sfft_batch_last_form(void) {
  std::lock_guard<std::mutex> g(g_mu);
  return g_last_form;
}

sfft_status sfft_plan_autotune(sfft_plan plan, int64_t nrhs, int use_cache, void* stream, double* best_us) {
  if (!plan) return sfft_rt_fail(SFFT_INVALID_ARG, "plan is null");
  if (nrhs < 1) return sfft_rt_fail(SFFT_INVALID_ARG, "nrhs must be >= 1");
  hipStream_t st = (hipStream_t)stream;
  const std::string key = tune_key(plan, nrhs);
  int sched = 0, rb = 0;
  std::string tiles;
  if (use_cache && tune_lookup(key, &sched, &rb, &tiles)) {
    if (plan->method == SFFT_SPLIT) plan->sched = sched;
    plan->rb_pref = rb;
    for (int l = 0; l < plan->d; ++l) plan->tile_mode[l] = l < (int)tiles.size() ? tiles[l] - '0' : 0;
    if (best_us) *best_us = -1.0;
    return SFFT_OK;
  }
  std::vector<std::pair<int, int>> cand;
  std::vector<int> scheds;
  if (plan->method == SFFT_SPLIT && plan->d > 2) scheds = {SFFT_SCHED_BREADTH, SFFT_SCHED_DEPTH, SFFT_SCHED_SLAB};
  else if (plan->method == SFFT_SPLIT && plan->d > 1) scheds = {SFFT_SCHED_BREADTH, SFFT_SCHED_DEPTH};
  else scheds = {plan->sched};
  const int rbmax = sfft_rt_leaf_rbmax(plan);
  for (int sc : scheds)
    for (int r = 1; r <= rbmax && (r == 1 || r <= 2 * nrhs - 1); r *= 2) cand.push_back({sc, r});
  const size_t vbytes = (size_t)(nrhs * plan->b * plan->s) * plan->esz;
  const int old_sched = plan->sched, old_rb = plan->rb_pref;
  int old_tiles[kMaxD];
  for (int l = 0; l < kMaxD; ++l) {
    old_tiles[l] = plan->tile_mode[l];
    plan->tile_mode[l] = 0;  // schedules and groupings are timed with the rule's widths
  }
  size_t wsmax = 0;
  for (int sc : scheds) {
    plan->sched = sc;
    const size_t w = sfft_rt_workspace_elems(plan, nrhs) * plan->esz;
    wsmax = w > wsmax ? w : wsmax;
  }
  plan->sched = old_sched;
  void *x = nullptr, *y = nullptr, *ws = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  sfft_status s = SFFT_OK;
  hipError_t he = hipMalloc(&x, vbytes);
  if (he == hipSuccess) he = hipMalloc(&y, vbytes);
  if (he == hipSuccess && wsmax) he = hipMalloc(&ws, wsmax);
  // a nonzero input (every byte 0x3c: normal numbers in FP32 and FP64)
  if (he == hipSuccess) he = hipMemsetAsync(x, 0x3c, vbytes, st);
  if (he == hipSuccess) he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  if (he != hipSuccess) s = sfft_rt_hip_fail(he, "autotune buffers");
  // each candidate: one warm-up apply, then three trials of `reps` applies
  // (reps sized so a trial lasts about 2 ms, at least 3), keeping the fastest
  // trial; the faster of the low-memory schedules (depth-first, the paper's
  // peak memory, and its slab form) wins unless breadth-first is more than 3%
  // faster
  double best = 1e300, best_depth = 1e300;
  int bs = old_sched, br = old_rb, bds = SFFT_SCHED_DEPTH, bdr = old_rb;
  auto time_reps = [&](int reps, double* us) -> sfft_status {
    he = hipEventRecord(e0, st);
    sfft_status r = SFFT_OK;
    for (int i = 0; i < reps && r == SFFT_OK; ++i) r = sfft_rt_apply_one(plan, x, y, nrhs, ws, wsmax, st);
    if (r != SFFT_OK) return r;
    if (he == hipSuccess) he = hipEventRecord(e1, st);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float ms = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    if (he != hipSuccess) return sfft_rt_hip_fail(he, "autotune timing");
    *us = 1e3 * ms / reps;
    return SFFT_OK;
  };
  // one candidate: a warm-up apply, then three trials of `reps` applies
  auto time_candidate = [&](double* cbest) -> sfft_status {
    sfft_status r = sfft_rt_apply_one(plan, x, y, nrhs, ws, wsmax, st);  // warm-up
    double est = 0.0;
    if (r == SFFT_OK) r = time_reps(1, &est);
    if (r != SFFT_OK) return r;
    int reps = est > 0.0 ? (int)(2000.0 / est) : 3;
    reps = reps < 3 ? 3 : (reps > 200 ? 200 : reps);
    *cbest = 1e300;
    for (int trial = 0; trial < 3 && r == SFFT_OK; ++trial) {
      double us = 0.0;
      r = time_reps(reps, &us);
      if (r == SFFT_OK && us < *cbest) *cbest = us;
    }
    return r;
  };
  for (auto& c : cand) {
    if (s != SFFT_OK) break;
    plan->sched = c.first;
    plan->rb_pref = c.second;
    double cbest = 1e300;
    s = time_candidate(&cbest);
    if (s != SFFT_OK) break;
    if (cbest < best) {
      best = cbest;
      bs = c.first;
      br = c.second;
    }
    if (c.first != SFFT_SCHED_BREADTH && cbest < best_depth) {  // the low-memory schedules
      best_depth = cbest;
      bds = c.first;
      bdr = c.second;
    }
  }
  if (s == SFFT_OK && bs == SFFT_SCHED_BREADTH && best_depth < 1e300 && best > 0.97 * best_depth) {
    bs = bds;
    br = bdr;
    best = best_depth;
  }
  // then, level by level, a fixed workgroup width for the strided passes
  // (levels 1..d-1; the last level is the leaf) against the rule, kept only
  // when more than 1% faster
  if (s == SFFT_OK) {
    plan->sched = bs;
    plan->rb_pref = br;
    for (int l = 0; l + 1 < plan->d && s == SFFT_OK; ++l) {
      if (!plan->ops[l]->strided_prep[1]) continue;  // the length has one width only
      int keep = 0;
      double lbest = best;
      for (int mode = 1; mode <= 2 && s == SFFT_OK; ++mode) {
        plan->tile_mode[l] = mode;
        double us = 1e300;
        s = time_candidate(&us);
        if (s == SFFT_OK && us < 0.99 * lbest) {
          lbest = us;
          keep = mode;
        }
      }
      plan->tile_mode[l] = keep;
      best = lbest;
    }
  }
  (void)hipStreamSynchronize(st);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (x) (void)hipFree(x);
  if (y) (void)hipFree(y);
  if (ws) (void)hipFree(ws);
  if (s != SFFT_OK) {
    plan->sched = old_sched;
    plan->rb_pref = old_rb;
    for (int l = 0; l < kMaxD; ++l) plan->tile_mode[l] = old_tiles[l];
    return s;
  }
  plan->sched = bs;
  plan->rb_pref = br;
  std::string tiles_out;
  for (int l = 0; l < plan->d; ++l) tiles_out.push_back((char)('0' + plan->tile_mode[l]));
  if (use_cache) tune_store(key, bs, br, tiles_out, best);
  if (best_us) *best_us = best;
  return SFFT_OK;
}

}  // extern "C"
