// Internal plan structure and runtime entry points shared by runtime.hip
// (plan creation, schedules, C ABI) and batch.hip (graph-batched multi-problem
// apply, autotuner). Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/sfft.h"
#include "axis_kernels.hpp"

constexpr int kMaxD = 6;

// Longest level a pencil kernel takes; a longer level is carried as several
// plan levels (below).
constexpr int64_t kMaxLevel = 2048;

// Gather of the caller's coefficients into the generator of the plan's levels
// when a level of size n = f_1 ... f_m (C order, so index i = sum_k i_k w_k
// with w_k = f_{k+1} ... f_m) is carried as m levels: entry (i - j) of a
// Toeplitz level is t(sum_k (i_k - j_k) w_k), an m-level Toeplitz operator
// whose generator at offsets (r_1, ..., r_m), |r_k| < f_k, is t(sum_k r_k w_k)
// (|sum_k r_k w_k| < n, so every offset is in the caller's array). The
// vectors keep their memory layout. Plan level q with offset index
// i_q (offset i_q - f_q + 1) reads the caller's array at
// cbase + sum_q i_q mult[q] within each block component.
struct Regather {
  int dq = 0;
  int64_t ext[kMaxD] = {0};   // 2 f_q - 1 offsets per plan level
  int64_t mult[kMaxD] = {0};  // caller-array stride per unit of i_q
  int64_t cbase = 0;          // caller-array offset of i = 0 (within a component)
  int64_t ncoef_in = 0;       // entries per block component: caller's array
  int64_t ncoef_out = 0;      // and the plan's generator
};

// A plan: level sizes, block size, dtype, method, schedule, FP64-generated
// symbols in the compute dtype and per-level twiddle tables (device memory
// owned by the plan), plus an optional workspace pool and profiling events.
struct sfft_plan_s {
  int d = 0;
  int64_t n[kMaxD] = {0};
  int user_d = 0;               // the caller's levels (size-1 levels are dropped from d, n)
  int64_t user_n[kMaxD] = {0};
  // levels longer than kMaxLevel split into several plan levels: the gather
  // of the caller's coefficients (creation and update), and the first plan
  // level of each caller level of size > 1
  bool regather = false;
  Regather rg;
  int eff_first[kMaxD] = {0};
  int b = 1;
  int dtype = SFFT_C64;
  int method = SFFT_SPLIT;
  int sched = SFFT_SCHED_BREADTH;
  int compressed = 0;
  int64_t max_nrhs = 1;
  int64_t s = 1;     // grid points
  size_t esz = 8;    // bytes per complex entry
  int64_t L[kMaxD];  // pencil length per level (n_l split, 2 n_l embed)
  const sfft::AxisOps* ops[kMaxD] = {nullptr};
  void* tw[kMaxD] = {nullptr};
  void* sym = nullptr;
  size_t sym_bytes = 0;
  int64_t sym_bs = 0;  // symbol entries per leaf branch prefix
  int64_t ntiles = 0;  // leaf tiles per component per rhs
  int64_t npen = 0;    // leaf pencils per component per rhs
  // block symmetry of the coefficients (0 none, 1 symmetric, 2 antisymmetric)
  // and the stored block components: comp_of[k] = a*b + c of stored component k
  int bsym = 0;
  int ns = 1;
  int comp_of[16] = {0};
  // mirrored symbol storage (compressed = 1): the declared per-(component,
  // level) parity [(a*b + c)*d + l] (checked against the coefficients at
  // creation and update) and, per stored component k, bit l of odd[k] set
  // when that component is odd along level l
  int64_t mst[kMaxD] = {0};
  int64_t mcomp = 0;
  // mirrored storage along the last level: mpair = 1 stores each parity's
  // half row in lane pairs (see k_scatter_mirror), mrow entries per row
  int mpair = 0;
  int64_t mrow = 0;
  int32_t parity[16 * kMaxD] = {0};
  uint8_t odd[16] = {0};
  // symbols of the conjugate transpose T^H (sfft_plan_enable_adjoint): the
  // same layout with component (a, c) holding conj of component (c, a), and
  // the odd-level bits of the component each stored one comes from
  void* sym_adj = nullptr;
  uint8_t odd_adj[16] = {0};
  // right-hand sides per leaf workgroup chosen by the autotuner (0: automatic)
  int rb_pref = 0;
  int tile_mode[kMaxD] = {0};  // strided passes per level: 0 rule, 1 full-size, 2 half-size workgroups
  size_t table_bytes = 0;
  std::mutex pool_mu;
  void* pool = nullptr;
  size_t pool_bytes = 0;
  // profiling hooks: event pairs around launches of the kinds in prof_mask
  // (records and the free list are guarded by prof_mu, so applies of one plan
  // from several host threads may profile at once)
  unsigned prof_mask = 0;
  std::mutex prof_mu;
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Rec> prof_recs;
  std::vector<hipEvent_t> prof_free;

  ~sfft_plan_s() {
    for (auto& r : prof_recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : prof_free) (void)hipEventDestroy(e);
    for (int l = 0; l < kMaxD; ++l)
      if (tw[l]) (void)hipFree(tw[l]);
    if (sym) (void)hipFree(sym);
    if (sym_adj) (void)hipFree(sym_adj);
    if (pool) (void)hipFree(pool);
  }
};

sfft_status sfft_rt_fail(sfft_status s, const std::string& msg);
sfft_status sfft_rt_hip_fail(hipError_t e, const char* what);
size_t sfft_rt_workspace_elems(const sfft_plan_s* p, int64_t nrhs);
sfft_status sfft_rt_apply_one(sfft_plan_s* p, const void* x, void* y, int64_t nrhs, void* ws, size_t ws_bytes,
                              hipStream_t st, bool adj = false);
int sfft_rt_leaf_rbmax(const sfft_plan_s* p);
// The kernels a leaf launch can use: one launch of its own, and the grouped
// launch's prep and launch functions (null where the length has none).
struct LeafSel {
  sfft::pass_fn single = nullptr;
  sfft::leaf_prep_fn prep = nullptr;
  sfft::leaf_group_fn group = nullptr;
};
// Arguments of level l's pass over nv vectors (whole vectors, one branch).
sfft::PassArgs sfft_rt_pass_args(const sfft_plan_s* p, int l, int64_t nv);
// Leaf arguments over branches 0 .. nq-1 (whole vectors).
sfft_status sfft_rt_leaf_args(const sfft_plan_s* p, const void* in, void* out, int64_t in_bs, int64_t nq,
                              int64_t nrhs, sfft::PassArgs* a, LeafSel* sel);
// Workspace entries of the breadth-first schedule (what grouped batches use).
size_t sfft_rt_breadth_workspace_elems(const sfft_plan_s* p, int64_t nrhs);
// drops cached graphs that reference the plan (called before it is freed)
void sfft_rt_forget_plan(const sfft_plan_s* p);

inline size_t sfft_rt_align256(size_t x) { return (x + 255) & ~size_t(255); }
