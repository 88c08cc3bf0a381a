/*
 * sfft.h -- C ABI of the split-FFT multilevel block-Toeplitz matrix-vector
 * product for AMD Instinct MI355X (gfx950).
 *
 * The operation (Siron & Molesky, "A Split Fast Fourier Transform Algorithm
 * for Block Toeplitz Matrix-Vector Multiplication", Algorithm 1 and its
 * statement y = T v): for a d-level block-Toeplitz matrix with b x b blocks on
 * the grid n_1 x ... x n_d,
 *
 *     y[a, i] = sum_{j in grid} sum_{c < b} t(i - j)[a, c] * x[c, j].
 *
 * SFFT_SPLIT evaluates it with the lazy-embedding / eager-projection split of
 * Section II (per level an even branch and a phase-shifted odd branch of the
 * unpadded vector, 2^d branch products with the parity parts T[bId] of the
 * embedded symbol, inverse transforms merged back level by level). SFFT_EMBED
 * evaluates the same product with the standard circulant embedding of every
 * level (vectors padded to 2n per level), the baseline the paper compares to.
 *
 * Layouts (C order, interleaved complex: re, im):
 *   coefficients  (b, b, 2n_1-1, ..., 2n_d-1) complex128; offset r_l is at
 *                 index r_l + n_l - 1 along level l (level 1 outermost).
 *   x, y          (nrhs, b, n_1, ..., n_d) of the plan's dtype.
 * All pointers passed to sfft_plan_create / sfft_apply / sfft_apply_multi are
 * DEVICE pointers unless marked "host". Streams are hipStream_t (NULL = the
 * null stream).
 *
 * Errors: every call returns an sfft_status; nothing is thrown across the
 * ABI. sfft_last_error() returns a message for the calling thread's last
 * failure. A HIP failure inside a call returns SFFT_HIP_ERROR.
 */
#ifndef SFFT_H
#define SFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sfft_plan_s* sfft_plan;

typedef enum {
  SFFT_OK = 0,
  SFFT_INVALID_ARG = 1,   /* null pointer, d < 1, n_l < 1, b not in {1..4}, bad enum, x aliases y,
                             short workspace, declared parity not held by the coefficients */
  SFFT_UNSUPPORTED = 2,   /* level size with a prime factor outside {2, 3, 5, 7}, more than 6 levels */
  SFFT_OUT_OF_MEMORY = 3, /* device allocation failed */
  SFFT_HIP_ERROR = 4      /* a HIP runtime call or kernel launch failed */
} sfft_status;

typedef enum {
  SFFT_C64 = 0,  /* complex64: FP32 arithmetic and accumulation, FP64-generated twiddles and symbols */
  SFFT_C128 = 1  /* complex128: FP64 throughout */
} sfft_dtype;

typedef enum {
  SFFT_SPLIT = 0, /* Algorithm 1: lazy embedding, eager projection */
  SFFT_EMBED = 1  /* standard multilevel circulant embedding (baseline) */
} sfft_method;

typedef enum {
  SFFT_SCHED_AUTO = 0,    /* depth-first (the paper's peak memory); sfft_plan_autotune may pick breadth-first */
  SFFT_SCHED_BREADTH = 1, /* all branches of a level per launch: workspace (2^d - 2) vectors */
  SFFT_SCHED_DEPTH = 2,   /* Algorithm 1's lazy order: workspace (d - 1) vectors, peak (d + 1) with x, y */
  SFFT_SCHED_SLAB = 3     /* d >= 3: Algorithm 1's order with levels 2..d over slabs of consecutive
                             level-1 indices, each slab's grandchildren small enough (about 48 MB
                             each; SFFT_SLAB_MB overrides) to stay in the memory-side cache between
                             launches: workspace one vector plus (d - 1) slab vectors; d <= 2 as DEPTH */
} sfft_schedule;

/* Per-(component, level) symmetry of the generator t, used to store the
 * symbol mirrored (Section II.C): EVEN means t(.., -r_l, ..)[a,c] = t(.., r_l, ..)[a,c],
 * ODD means t(.., -r_l, ..)[a,c] = -t(.., r_l, ..)[a,c] (so the r_l = 0 plane is 0). */
typedef enum { SFFT_PARITY_NONE = 0, SFFT_PARITY_EVEN = 1, SFFT_PARITY_ODD = 2 } sfft_parity;

typedef struct {
  int d;
  int64_t n[8];
  int b;
  int dtype;
  int method;
  int schedule;            /* the schedule sfft_apply uses */
  int compressed;          /* 1 when the symbol is stored mirrored */
  int64_t max_nrhs;
  size_t symbol_bytes;     /* device bytes held by the plan's symbols */
  size_t table_bytes;      /* device bytes of twiddle tables */
  size_t workspace_bytes;  /* sfft_workspace_size at max_nrhs */
  int64_t vector_elems;    /* b * prod(n_l): entries of one right-hand side */
  int block_symmetry;      /* 0, or 1 / 2 when t[a,c] = t[c,a] / -t[c,a] at every offset:
                              the symbol then stores the b(b+1)/2 components a <= c */
  size_t adjoint_symbol_bytes; /* device bytes of the T^H symbols (0 until sfft_plan_enable_adjoint) */
  int tile_mode[8];        /* per level, the strided passes' workgroup width: 0 by rule (128 lanes
                              below 2048 workgroups, else 256), 1 always 256, 2 always 128 lanes
                              (set by sfft_plan_autotune; 0 for levels of size 1) */
  int64_t mirror_row;      /* mirrored storage: stored entries along the last level (n_d + 1, or
                              n_d + E/2 where the leaf reads lane pairs, E its entries per lane);
                              symbol_bytes = components x prod_{l<d}(n_l + 1) x mirror_row x dtype
                              size. 0 without mirrored storage */
  int plan_d;              /* levels the plan runs: d without its levels of size 1, a level above
                              2048 counted as the two or more levels that carry it */
  int64_t plan_n[8];       /* their sizes, outermost first */
  int64_t pencil_len[8];   /* per plan level, the transform length (n_l split, 2 n_l embedding) */
  int radix[8][8];         /* per plan level, the radices of its pass kernels, outermost stage
                              first, 0-terminated */
  int leaf_radix[8];       /* the radices of the leaf kernel (innermost plan level), 0-terminated */
  size_t peak_bytes;       /* device bytes of one apply at max_nrhs, as modelled: symbols (and
                              adjoint symbols when enabled), twiddle tables, workspace, x and y */
} sfft_info;

/* Build a plan and its Fourier-space symbols.
 *
 * Section II.B / II.C: the embedded generator (every level extended n -> 2n,
 * pad entry 0) is transformed in FP64 on the GPU, scaled by 2^-d / prod(n_l),
 * split into the 2^d parity parts T[bId] (SFFT_SPLIT) or kept whole
 * (SFFT_EMBED) and stored in the compute dtype.
 *
 *   out       host: receives the plan handle (NULL on failure).
 *   d         levels, 1 <= d <= 6.
 *   n         host: d level sizes with no prime factor above 7. A level of
 *             size 1 (offset 0 only) is dropped internally; at least one level
 *             must be larger (else SFFT_UNSUPPORTED). A level above 2048 is
 *             carried as two or more plan levels of at most 2048 each (the
 *             multilevel structure of the introduction: a Toeplitz level of
 *             size f_1 f_2 is a two-level Toeplitz operator with generator
 *             t(r_1 f_2 + r_2)); the coefficients are gathered into that
 *             generator on the device (scratch of b*b*prod(2f_q - 1) complex128
 *             entries during the call), the vectors keep their layout, and
 *             sfft_apply_subtree's k and the schedules count plan levels.
 *             SFFT_UNSUPPORTED if the plan levels number more than 6, or with
 *             a parity mask on a split plan (mirrored storage needs level
 *             sizes up to 2048).
 *   b         block size, 1 <= b <= 4.
 *   coeffs    device, complex128 (b, b, 2n_1-1, ..., 2n_d-1); read during the
 *             call only (the stream is synchronised before return, the caller
 *             may free it afterwards).
 *   dtype     SFFT_C64 or SFFT_C128.
 *   method    SFFT_SPLIT or SFFT_EMBED.
 *   parity    host, NULL or b*b*d sfft_parity values [(a*b + c)*d + l]: when
 *             every entry is EVEN or ODD and method is SFFT_SPLIT, the symbol
 *             is stored mirrored (about prod(n_l + 1) per component instead
 *             of 2^d prod(n_l)). The declared symmetry is checked exactly
 *             against the coefficients (SFFT_INVALID_ARG on a mismatch).
 *   max_nrhs  largest nrhs a later apply may use (sizes sfft_plan_info only).
 *   schedule  sfft_schedule.
 *   stream    hipStream_t for the generation kernels.
 * The plan owns its device memory and changes only through sfft_plan_update;
 * one plan may be applied concurrently on several streams with distinct
 * workspaces. */
sfft_status sfft_plan_create(sfft_plan* out, int d, const int64_t* n, int b, const void* coeffs,
                             int dtype, int method, const int32_t* parity, int64_t max_nrhs,
                             int schedule, void* stream);

/* Regenerates the plan's symbols (Section II: the FFT of the embedded
 * generator, split by parity per level) from new coefficients in place, so a
 * plan and its memory serve another Toeplitz matrix of the same shape: sizes,
 * buffers, workspace needs and batched-apply graphs that hold the plan stay
 * valid, and nothing is allocated beyond the generation scratch (ordered on
 * `stream`).
 *   coeffs  device, complex128, the layout of sfft_plan_create; its block
 *           symmetry (every pair t[a,c] = t[c,a], or every pair
 *           t[a,c] = -t[c,a], or neither) must equal the plan's
 *           (sfft_info.block_symmetry), and a mirrored plan's coefficients
 *           must keep the parity it was created with (checked exactly), else
 *           SFFT_INVALID_ARG and the plan is unchanged.
 *   stream  hipStream_t for the generation kernels, synchronised before
 *           return. Every earlier use of the plan (applies on any stream) must
 *           be ordered before the work on `stream`: the symbols are
 *           overwritten in place.
 * Errors: SFFT_INVALID_ARG (null plan or coeffs, other block symmetry),
 * SFFT_OUT_OF_MEMORY / SFFT_HIP_ERROR (generation scratch or kernels; the
 * symbols are then undefined until a successful update). */
sfft_status sfft_plan_update(sfft_plan plan, const void* coeffs, void* stream);

/* Device bytes of workspace sfft_apply needs for nrhs >= 0 right-hand sides
 * (0 for nrhs = 0). */
sfft_status sfft_workspace_size(sfft_plan plan, int64_t nrhs, size_t* bytes);

/* y = T x for nrhs right-hand sides (Algorithm 1, or the embedding baseline).
 *   nrhs       >= 0; nrhs = 0 is an empty batch: SFFT_OK, nothing is touched
 *              (x, y and workspace may then be NULL).
 *   x, y       device (nrhs, b, n...) of the plan dtype; y must not overlap x.
 *   workspace  device, at least sfft_workspace_size bytes, 256-byte aligned,
 *              caller owned; NULL makes the plan allocate (and keep) its own,
 *              which is then not safe for concurrent applies of one plan.
 *   stream     hipStream_t; the call only enqueues work (asynchronous). */
sfft_status sfft_apply(sfft_plan plan, const void* x, void* y, int64_t nrhs, void* workspace,
                       size_t ws_bytes, void* stream);

/* sfft_apply for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc. The
 * same product as sfft_apply (same kernels and schedule), with the workspace
 * taken from a static device array of the library (128 MiB per device, held
 * until the process ends) instead of a caller buffer or a plan-owned pool; the
 * call allocates nothing and records no profiling events.
 *   Errors: SFFT_INVALID_ARG when the workspace sfft_workspace_size reports for
 *   nrhs exceeds 128 MiB (nothing is launched), and as sfft_apply otherwise.
 * Every call on one device shares that device's array: calls that overlap on
 * one device (other host threads, or other streams not ordered after this
 * one) race on it. The array needs no clearing (every pass writes before it
 * reads). The current device must be the plan's device. */
sfft_status sfft_apply_noalloc(sfft_plan plan, const void* x, void* y, int64_t nrhs, void* stream);

/* Out-of-core product for vectors that stay in host memory (the paper's
 * remark on larger systems: the input pre-partitioned into nearly independent
 * even and odd parts). After the level-1 split the two children are
 * independent products over levels 2..d, and every level-1 frequency index
 * of a child is independent of the others, so the product runs as
 *   1. column slabs of x to the device, level-1 forward pass (both children),
 *      children back to the host workspace;
 *   2. per child, slabs of consecutive level-1 indices to the device, levels
 *      2..d depth-first there (the plan's symbols stay on the device), back;
 *   3. column slabs of both children to the device, level-1 inverse pass and
 *      merge, y back to the host.
 * The device holds the plan and slabs only. When the budget holds two slab
 * buffers, consecutive slabs alternate between them on `stream` and an
 * internal stream, so one slab's copies overlap the other's kernels. Results
 * equal sfft_apply's depth-first product bit for bit (same kernels, same
 * per-pencil work).
 *   x_host, y_host  host (nrhs, b, n...) of the plan dtype, preferably pinned
 *                   (hipHostMalloc) so the copies run asynchronously.
 *   host_ws         host, 2 * nrhs * b * prod(n) entries: the two children
 *                   (pinned too, preferably).
 *   device_ws       device, its size is the budget: sfft_ooc_sizes tells the
 *                   bytes a budget actually uses (SFFT_INVALID_ARG when one
 *                   slab does not fit).
 * Split plans with d >= 2 only (SFFT_UNSUPPORTED otherwise). Synchronous:
 * returns when y_host is complete. */
sfft_status sfft_ooc_sizes(sfft_plan plan, int64_t nrhs, size_t device_budget, size_t* host_ws_bytes,
                           size_t* device_ws_bytes);
sfft_status sfft_apply_ooc(sfft_plan plan, const void* x_host, void* y_host, int64_t nrhs, void* host_ws,
                           size_t host_ws_bytes, void* device_ws, size_t device_ws_bytes, void* stream);

/* One device's share of a product split over 2^k devices by branch. After
 * the splits of levels 1..k the 2^k branches are independent (Section II's
 * opening remarks on several devices: by linearity a branch may run on to a
 * chosen termination point instead of merging): the share of branch `prefix`
 * forms, along each level
 * l <= k, only the child whose parity is bit l-1 of prefix, runs the subtree
 * below level k depth-first, and merges back along levels k..1 with that child
 * alone. The 2^k shares of one x sum to T x (one sum-reduce of y across
 * devices). k = 0 is the whole depth-first product.
 *   k          0 <= k <= d - 1 (the plan's d, levels of size 1 dropped).
 *   prefix     < 2^k; bit l-1 is the parity along level l.
 *   x, y       device (nrhs, b, n...) of the plan dtype; y must not overlap x.
 *   workspace  device, at least sfft_workspace_size_subtree bytes
 *              ((d - 1 - k) vectors), caller owned, not NULL when that is > 0.
 * Split plans only (SFFT_UNSUPPORTED for the embedding baseline); general and
 * mirrored symbols. Asynchronous on `stream`; allocates nothing. */
sfft_status sfft_workspace_size_subtree(sfft_plan plan, int k, int64_t nrhs, size_t* bytes);
sfft_status sfft_apply_subtree(sfft_plan plan, int k, uint32_t prefix, const void* x, void* y, int64_t nrhs,
                               void* workspace, size_t ws_bytes, void* stream);

/* The conjugate transpose, y = T^H x: T^H is block Toeplitz with generator
 * t^H(r) = t(-r)^H, whose embedded symbol is the conjugate transpose of T's at
 * every bin (Section II's embedding with the generator reversed), so the
 * plan's parity parts T[bId] serve it conjugated and transposed.
 * sfft_plan_enable_adjoint allocates and fills these symbols once (the
 * plan's symbol size again; synchronises `stream`); sfft_plan_update refreshes
 * them. sfft_apply_adjoint takes the arguments and workspace of sfft_apply,
 * allocates nothing, and returns SFFT_INVALID_ARG before the adjoint is
 * enabled. */
sfft_status sfft_plan_enable_adjoint(sfft_plan plan, void* stream);
sfft_status sfft_apply_adjoint(sfft_plan plan, const void* x, void* y, int64_t nrhs, void* workspace,
                               size_t ws_bytes, void* stream);

/* Several independent products in one call: problem i is plans[i] applied to
 * x[i] -> y[i] with nrhs[i] right-hand sides (host arrays of device
 * pointers; workspace at least sfft_workspace_size_multi bytes, problem i at
 * the 256-byte aligned offset of the preceding problems' sizes; no problem's
 * y may overlap any problem's x or y). The batch is captured into a HIP graph
 * and replayed by one graph launch on `stream`, in one of two forms with
 * bit-identical results: per-problem chains (every problem's launches in its
 * own schedule on its own forked stream, so problems run side by side) or
 * grouped lanes (problems with equal level lengths form a lane on its own
 * forked stream; step k of every member's breadth-first schedule in stage k,
 * the entries of one kernel in one launch: 2d - 1 stages per lane). The first
 * call with an argument set captures both, replays each on `stream` a few
 * times (waiting for them: that call blocks the host for some milliseconds)
 * and keeps the faster; SFFT_BATCH_MODE=chains or =grouped in the environment
 * captures only that form. The instantiated graph is cached for the same
 * arguments and dropped when one of its plans is destroyed. SFFT_NO_GRAPH=1
 * issues the problems one after another instead. A problem with nrhs[i] = 0
 * is skipped (its x[i], y[i] may be NULL). INVALID_ARG when x[i] == y[i]. */
sfft_status sfft_workspace_size_multi(int nprob, const sfft_plan* plans, const int64_t* nrhs,
                                      size_t* bytes);
sfft_status sfft_apply_multi(int nprob, const sfft_plan* plans, const void* const* x,
                             void* const* y, const int64_t* nrhs, void* workspace, size_t ws_bytes,
                             void* stream);
/* Form of the graph that the last sfft_apply_multi graph launch (any thread)
 * replayed: 0 per-problem chains, 1 grouped lanes, -1 none yet. */
int sfft_batch_last_form(void);

/* Independent products issued in one call without a graph, each with its own
 * caller workspace: problem i is plans[i] applied to x[i] -> y[i] (nrhs[i]
 * right-hand sides, workspaces[i] of ws_bytes[i] bytes, NULL when 0 is
 * needed), on internal streams forked from `stream` and joined back to it, so
 * the problems' kernels overlap and later work on `stream` sees every result.
 * For loops that change the set of problems every call (a serving step), where
 * a cached graph would rarely be replayed. status (host, nprob entries)
 * receives each problem's own result; a failing problem does not stop the
 * others. Returns SFFT_OK unless the call itself is malformed or a fork/join
 * fails. */
sfft_status sfft_apply_each(int nprob, const sfft_plan* plans, const void* const* x, void* const* y,
                            const int64_t* nrhs, void* const* workspaces, const size_t* ws_bytes, void* stream,
                            sfft_status* status);

sfft_status sfft_plan_info(sfft_plan plan, sfft_info* info);

/* One step of independent Arnoldi processes (Krylov chains of matvecs, the
 * iterative-solver setting of the paper's introduction). For every job the
 * new vector w (typically T v_{m-1}) is orthogonalised against the basis
 * v_0..v_{m-1} (assumed orthonormal) by classical Gram-Schmidt, with a second
 * pass when the first leaves less than half of ||w||^2 (the Kahan-Parlett
 * "twice is enough" test), then normalised:
 *     hcol[i] = <v_i, w> (passes summed), hcol[m] = ||w||, vout = w/||w||.
 * m = 0 only normalises (the start vector). Reductions accumulate in FP64 in
 * a fixed order and the test uses only the job's own sums, so results are
 * bitwise independent of the other jobs.
 * All pointers are device pointers; vectors are of `dtype` (one dtype per
 * call); hcol is complex128. scratch: sfft_arnoldi_scratch_size bytes. */
typedef struct {
  const void* V;   /* basis v_0..v_{m-1}, v_i at V + i*ldv entries */
  int64_t ldv;     /* entries between basis vectors (>= n) */
  int64_t m;       /* basis vectors, 0 <= m <= 64 */
  void* w;         /* n entries, overwritten by its orthogonalised form */
  void* vout;      /* receives w / ||w|| (may be w or the basis slot v_m) */
  int64_t n;       /* entries per vector */
  void* hcol;      /* m + 1 complex128 entries */
} sfft_arnoldi_job;

sfft_status sfft_arnoldi_scratch_size(int njobs, const sfft_arnoldi_job* jobs, size_t* bytes);
sfft_status sfft_arnoldi_step_multi(int njobs, const sfft_arnoldi_job* jobs, int dtype, void* scratch,
                                    size_t scratch_bytes, void* stream);

/* Restarted GMRES(m) for the scattering operator A = I - diag(chi) T (T the
 * plans' block-Toeplitz matrix, chi a per-entry susceptibility, typically
 * nonzero on a small region): the Krylov solve whose matvecs the split
 * product accelerates (the paper's introduction). Mixed-precision iterative
 * refinement: every cycle runs up to m Arnoldi steps with products of `lo`
 * (complex64 or complex128), each step's Hessenberg column comes back to the
 * host for Givens rotations, the correction is added to x in FP64, and the
 * true residual b - A x is recomputed in FP64 with `hi` (a complex128 plan of
 * the same operator; it may be lo itself when lo is complex128). Stops when
 * ||b - A x|| <= tol ||b|| or after max_cycles cycles.
 *   chi, rhs  device complex128 (b, n_1, ..., n_d): the diagonal of chi and b.
 *   x         device complex128 (b, n...): the initial guess on entry, the
 *             solution on return.
 *   m         Krylov steps per cycle, 1..64.
 *   workspace device, sfft_gmres_workspace_size bytes; nothing is allocated.
 *   stream    every kernel runs on it; the call returns when the solve is done
 *             (it synchronises after each Arnoldi step to read H).
 *   info      host, may be NULL: cycles, products and the final FP64 relative
 *             residual (recomputed, not estimated). */
typedef struct {
  int64_t cycles;                /* restart cycles run */
  int64_t matvecs;               /* products with T in lo's dtype */
  int64_t fp64_matvecs;          /* products with T in FP64 (true residuals) */
  double rel_residual;           /* ||b - A x|| / ||b||, FP64, at return */
  double rel_residual_estimate;  /* the last inner least-squares estimate */
  int converged;                 /* rel_residual <= tol */
} sfft_gmres_info;

sfft_status sfft_gmres_workspace_size(sfft_plan lo, sfft_plan hi, int m, size_t* bytes);
sfft_status sfft_gmres_solve(sfft_plan lo, sfft_plan hi, const void* chi, const void* rhs, void* x, int m,
                             int max_cycles, double tol, void* workspace, size_t ws_bytes, void* stream,
                             sfft_gmres_info* info);

/* Times the plan's candidate schedules (breadth-first and depth-first for
 * SFFT_SPLIT with d > 1, and the slab form for d > 2; a low-memory schedule
 * is kept unless breadth-first is more than 3% faster) and leaf
 * right-hand-side groupings (1, 2, 4, 8 per
 * workgroup, within the kernel's limit) at nrhs right-hand sides on `stream`,
 * and keeps the fastest in the plan (sfft_workspace_size follows the chosen
 * schedule); then, level by level, the strided passes' workgroup width (256
 * or 128 lanes, where the length has both) against the built-in rule,
 * keeping a fixed width only when it is more than 1% faster
 * (sfft_info.tile_mode). With use_cache != 0 a result stored for the same device,
 * method, dtype, block size, grid, storage and nrhs in the JSON-lines file
 * named by SFFT_TUNE_CACHE (default $HOME/.cache/sfft_autotune.jsonl) is
 * reused without timing, and new results are appended to it. Allocates and
 * frees its own scratch vectors; must not run concurrently with applies of
 * the same plan. best_us (may be NULL) receives the best time in
 * microseconds per apply, or -1 when the cache answered. */
sfft_status sfft_plan_autotune(sfft_plan plan, int64_t nrhs, int use_cache, void* stream, double* best_us);

/* Kernel classes for the profiling hooks. */
typedef enum {
  SFFT_KIND_FORWARD = 0, /* FWD2 passes: FFT along a level + phase split */
  SFFT_KIND_LEAF = 1,    /* last level: FFT, block product, iFFT, merge */
  SFFT_KIND_INVERSE = 2, /* INV2 passes: iFFT along a level + merge */
  SFFT_KIND_COPY = 3     /* embedding baseline's pad and projection */
} sfft_kernel_kind;

/* Bracket every later launch of the kinds set in mask (bit k = kind k) with a
 * pair of HIP events recorded on the apply stream; mask 0 stops recording.
 * Records accumulate until read with reset (about 2 events per launch);
 * concurrent applies of one plan may record (the record list is locked), but
 * enabling or disabling while applies run races with them. Launches inside
 * sfft_apply_multi's captured graphs are not recorded. */
sfft_status sfft_profile_enable(sfft_plan plan, unsigned mask);
/* Waits for the recorded events of one kind and returns their summed
 * duration in milliseconds and the launch count; reset != 0 clears them. */
sfft_status sfft_profile_read(sfft_plan plan, int kind, double* total_ms, int64_t* launches, int reset);
/* Frees the plan and its device memory (hipFree waits for the device work in
 * flight) and drops the batch graphs that hold it. SFFT_INVALID_ARG for a
 * null plan. */
sfft_status sfft_plan_destroy(sfft_plan plan);

const char* sfft_status_string(sfft_status s);
/* Message of the calling thread's last failed call ("" if none). */
const char* sfft_last_error(void);
/* Kernels for pencil length L: 1 when length-specialised kernels are built
 * (register-resident radix plans), 2 when L is served by the runtime-length
 * kernels (2 <= L <= 4096 with prime factors in {2, 3, 5, 7}: pencil tiles
 * staged whole in LDS), 0 otherwise. */
int sfft_length_supported(int64_t L);

#ifdef __cplusplus
}
#endif

#endif /* SFFT_H */
