/*
 * rrq.h - C ABI of the MI355X (gfx950) library for recursive reduction quadrature (RRQ):
 * assembly of the sparse near-field quadrature-correction matrix of the Laplace single-layer
 * (S), double-layer (D) and normal-derivative (S', D') potentials on quadrilateral patches.
 *
 * The operation is the one stated as the input/output of the algorithm in Sec. 4 of
 * Jiang & Zhu, "Recursive reduction quadrature for the evaluation of Laplace layer potentials
 * in three dimensions": patches with collocation nodes and boundary-edge nodes plus targets
 * go in; with Step 2 skipped as in the remark that follows the algorithm, the library returns
 * for every (target, near patch) pair the row of weights [w^T(x) A^+]_0 that maps nodal
 * densities to the potential at the target, for S (Theorem thm:slpreduction), D
 * (Lemma lem:dlpreduction, eq. wlmdef), S' (Sec. 3.6) and D' (Sec. 3.7).  With
 * RRQ_F_CORRECTION the smooth-rule weights K(x, r_j) w_j are subtracted (the splitting
 * D = D_smooth + D_RRQ of eq. dlpsplitting), giving the sparse correction matrix.
 *
 * Conventions
 *  - Pointers are DEVICE pointers unless a comment says HOST.  Arrays of 3-vectors are
 *    structure-of-arrays: x[0..n), y[0..n), z[0..n) at xyz, xyz + n, xyz + 2n.
 *  - Patch P has order q_P (q_P x q_P tensor Gauss-Legendre nodes; basis order p = q_P),
 *    nodes node_off[P] .. node_off[P+1] (node index a*q + b, parameter v = t_a, u = t_b), and
 *    4 edges ordered counter-clockwise about the outward normal, each with ptilde_P =
 *    2 q_P samples at increasing Gauss-Legendre parameters, stored at edge_off[P] + e*ptilde
 *    + i.  Neighbouring patches are expected to share edge curves.
 *  - Supported orders q: 4, 5, 6, 8, 10.  Other orders return RRQ_ERR_UNSUPPORTED.
 *  - Near list: CSR by target (near_ptr[T+1], near_patch[nnz]).  Weight blocks are stored
 *    target-major in near-list order: the block of pair k occupies [pair_off[k],
 *    pair_off[k+1]) with pair_off[k+1] - pair_off[k] = q_P^2, entry j = node j of patch P.
 *  - All calls are asynchronous on the caller's HIP stream (hipStream_t passed as void*;
 *    NULL = the default stream) unless noted.  Argument errors are detected on the host and
 *    returned before any launch.  Launch errors return RRQ_ERR_DEVICE.  No exception crosses
 *    the ABI.
 *  - A plan owns its device memory (maps, edge tables, frames); the caller owns every other
 *    buffer.  A plan may be used from several streams at once for assembly; refit and
 *    destroy must not overlap other calls on the same plan.
 */
#ifndef RRQ_H
#define RRQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RRQ_OK = 0,
  RRQ_ERR_ARG = -1,         /* invalid argument (null pointer, bad size, bad option, a near
                               list / self index / target outside its range)               */
  RRQ_ERR_DEVICE = -2,      /* a HIP call or kernel launch failed                           */
  RRQ_ERR_OOM = -3,         /* device allocation failed                                     */
  RRQ_ERR_ILLCONDITIONED = -4, /* rrq_plan_patch_flags: some patch fit is flagged (the plan
                               still produces weights for it)                               */
  RRQ_ERR_UNSUPPORTED = -5, /* order, size or option outside what this build supports       */
  RRQ_ERR_BUFFER = -6,      /* a caller buffer is too small                                 */
  RRQ_ERR_NONFINITE = -7    /* the call wrote NaN or Inf outputs (counted in rrq_stats and
                               marked in the per-pair flags)                                */
} rrq_status;

/* kernel mask bits */
enum { RRQ_K_S = 1, RRQ_K_D = 2, RRQ_K_SP = 4, RRQ_K_DP = 8, RRQ_K_ALL = 15 };

/* assembly flags */
enum {
  RRQ_F_CORRECTION = 1, /* subtract the smooth rule K(x, r_j) w_j (self node skipped)        */
  RRQ_F_ONSURF_PV = 2,  /* self targets: principal value for D and S' (else exterior limit) */
  RRQ_F_PLAIN = 8,      /* one workgroup per pair (reference form) instead of the batched form */
  RRQ_F_LEARNED = 16    /* batched form with the learned Newton initial guess (needs a model) */
};

typedef struct rrq_plan rrq_plan;

typedef struct {
  int32_t npatch;
  const int32_t* order_host; /* HOST [P] order q_P of each patch                          */
  const int32_t* order;      /* [P] same, on the device                                    */
  const int64_t* node_off;   /* [P+1]                                                      */
  const double* node_xyz;    /* [3][N] node coordinates                                    */
  const double* node_nrm;    /* [3][N] unit outward normals                                */
  const double* node_wt;     /* [N] smooth-rule weights (GL weights times area element)    */
  const int64_t* edge_off;   /* [P+1] = prefix sum of 4 * ptilde_P                         */
  const double* edge_xyz;    /* [3][E] edge samples                                        */
  int64_t nnode;             /* N */
  int64_t nedge;             /* E */
} rrq_surface;

typedef struct {
  int64_t ntarget;           /* T */
  int64_t nnz;               /* number of near pairs                                       */
  const double* xyz;         /* [3][T] target points                                       */
  const double* nrm;         /* [3][T] target unit normals nu' (used by S' and D')         */
  const int32_t* self_patch; /* [T] patch whose node the target is, or -1                  */
  const int32_t* self_node;  /* [T] local node index within self_patch, or -1              */
  const int64_t* near_ptr;   /* [T+1] CSR row pointer                                      */
  const int32_t* near_patch; /* [nnz] near patches of each target                          */
} rrq_targets;

typedef struct {
  double rho_far;       /* Bernstein radius above which an edge uses the plain GL rule;
                           <= 0 selects 10^(8/ptilde).  Values above that default for an
                           order present in the surface return RRQ_ERR_UNSUPPORTED (the
                           graded-panel capacity of the near-edge kernels is sized for it)  */
  double newton_tol;    /* Newton step tolerance (relative); <= 0 selects 1e-14             */
  int32_t newton_maxit; /* <= 0 selects 60                                                  */
  int32_t tile_targets; /* batched form: targets per workgroup tile (4 or 8); <= 0 = 4
                           until rrq_autotune picks one                                     */
  int32_t grid;         /* batched form: persistent workgroups per launch; <= 0 = 2048
                           until rrq_autotune picks one                                     */
  int32_t ls_unweighted; /* 0: least-squares rows weighted by sqrt(w_a w_b), the tensor GL
                           parameter weights (default); 1: unit row weights                 */
  int32_t ptilde_factor; /* edge samples per edge = ptilde_factor * q; 0 or 2 (the only
                           supported value; the paper's "2p"), else RRQ_ERR_UNSUPPORTED     */
  int32_t u_rule;       /* Dirac-string direction u of a pair: 0 = the target normal for a
                           self target, else +-normal of the nearest node pointing to the
                           target (the only supported rule), else RRQ_ERR_UNSUPPORTED       */
} rrq_options;

typedef struct {
  int64_t pairs;          /* pairs assembled                                               */
  int64_t near_edges;     /* (pair, edge) combinations integrated by singularity swap      */
  int64_t newton_iters;   /* total Newton iterations                                       */
  int64_t newton_fail;    /* edges whose Newton solve did not converge (plain rule used)   */
  int64_t learned_accept; /* edges whose learned initial guess was accepted                */
  int64_t newton_max;     /* largest iteration count of one edge                           */
  double kernel_ms;       /* device time of the pair kernels of this call (the per-pair
                             kernel of the plain form or the tile kernels of the batched form;
                             binning, the root pre-pass and the near-edge moment pre-pass
                             excluded), from HIP events on the call's stream                */
  int64_t newton_wave_iters; /* batched form: sum over wavefronts of the root pre-pass of
                             the largest iteration count among the wavefront's lanes (the
                             SIMD cost of the Newton solves)                               */
  int64_t panel_overflow; /* near edges whose graded panels exceeded the kernel's capacity
                             (the deepest panels, nearest the root, were dropped)           */
  int64_t nonfinite;      /* NaN or Inf outputs written (weights or pair potentials)        */
  int64_t flagged_pairs;  /* pairs with a non-zero flag word (see rrq_assemble)             */
  uint32_t invalid;       /* device check of the inputs: 1 near list, 2 self indices,
                             4 pair offsets or output length, 8 non-finite target; 0 = ok   */
  double order_kernel_ms[5]; /* batched form: device time of the tile kernel of each order
                             (4, 5, 6, 8, 10; 0 for absent orders), from HIP events        */
  int64_t newton_slots;   /* batched form: (pair, edge) slots whose Newton solve ran         */
  int64_t newton_over[5]; /* of those, the ones that took more than 2, 4, 6, 8 and 12
                             iterations (the tail of the iteration distribution)           */
} rrq_stats;

/* Create a plan for a surface: allocates the per-patch frames, coefficient maps and edge
 * tables, then computes them (Steps 1-3: source-only) on `stream`.  `opts` may be NULL. */
rrq_status rrq_plan_create(const rrq_surface* surf, const rrq_options* opts, void* stream,
                           rrq_plan** out);

/* Recompute the source-only data for a surface with the same patch count and orders
 * (new node/edge coordinates) into the plan's existing buffers.  Allocates nothing. */
rrq_status rrq_plan_refit(rrq_plan* plan, const rrq_surface* surf, void* stream);

rrq_status rrq_plan_destroy(rrq_plan* plan);

/* Conditioning of each patch's weighted least-squares fits (Steps 1-2; the study of the
 * system matrix in Sec. 5): cond[2P'] = ||A_w||_F ||A_w^+||_F, the Frobenius-norm condition
 * number of the weighted DLP system A_w (4q^2 x 4n_p, eq. dlpdensitylinearsystem2) of patch
 * P', with A_w^+ taken from the computed solutions; cond[2P'+1] the same for the SLP system
 * (q^2 x n_p, eq. slpdensitylinearsystem).  Each bounds the 2-norm condition number of its
 * weighted system from above, by at most the system's rank (4 n_p, resp. n_p) times it.  The
 * fits still produce maps whatever the value; a caller flags patches against its own
 * threshold (near 1/eps the fitted density loses accuracy).  cond is a HOST array of 2P doubles, filled from the last plan_create or
 * plan_refit; the call synchronises `stream`. */
rrq_status rrq_plan_fit_condition(const rrq_plan* plan, double* cond, void* stream);

/* Flags of the source-only data of every patch (Steps 1-2), into host_flags[P] (HOST): bit 1
 * = the DLP fit's condition estimate (rrq_plan_fit_condition) exceeds max_cond, bit 2 = the
 * SLP fit's does, bit 4 = the patch's frame, local geometry, maps or edge tables hold a NaN
 * or Inf.  max_cond <= 0 selects 1e9 (above it the fit's rounding can exceed about 1e-7 of
 * the density; the paper's conditioning study of Sec. 5 reaches 1/eps at p = 26).  Returns
 * RRQ_ERR_ILLCONDITIONED if any patch is flagged, RRQ_OK otherwise; flagged patches still
 * produce weights.  Synchronises `stream`; allocates and frees a small device buffer. */
rrq_status rrq_plan_patch_flags(const rrq_plan* plan, double max_cond, int32_t* host_flags,
                                void* stream);

/* Number of weights per kernel that rrq_assemble writes for this near list: the sum of q_P^2
 * over the near pairs, into *nweights (HOST).  Checks the near list on the host (row pointer
 * from 0 to nnz and non-decreasing, patch indices in range) and returns RRQ_ERR_ARG if it is
 * not valid.  Copies near_ptr and near_patch to the host: synchronous. */
rrq_status rrq_weights_size(const rrq_plan* plan, const rrq_targets* tg, int64_t* nweights,
                            void* stream);

/* Bytes of caller-provided device workspace that rrq_assemble needs for this near list. */
rrq_status rrq_workspace_size(const rrq_plan* plan, const rrq_targets* tg, size_t* bytes);

/* pair_off[nnz+1] (device) = prefix sum of q_P^2 over the near list (the output offset of
 * every pair's weight block).  `workspace` is the rrq_assemble workspace (its scan partials
 * are used).  The targets, near list and self indices are first checked on the device
 * (near_ptr from 0 to nnz and non-decreasing, near_patch in [0, P), self_patch in [-1, P),
 * self_node among the self patch's nodes, finite target points and normals).  Asynchronous;
 * if `nweights` (HOST) is non-NULL the call synchronises the stream, returns RRQ_ERR_ARG
 * before computing anything if the check failed, and returns there the total number of
 * weights per kernel.  Asynchronously, a failed check makes the call's kernels do nothing. */
rrq_status rrq_pair_offsets(const rrq_plan* plan, const rrq_targets* tg, int64_t* pair_off,
                            void* workspace, size_t workspace_bytes, int64_t* nweights,
                            void* stream);

/* Assemble the weight blocks of every near pair.  out_* are device arrays of out_len doubles
 * each (NULL for a kernel not in kmask); out_len must be at least the number of weights
 * (rrq_weights_size).  pair_off from rrq_pair_offsets.  pair_flags (device, [nnz], may be
 * NULL) receives one flag word per pair: 1 = the Newton solve of one of its edges did not
 * converge (that edge used the plain Gauss-Legendre rule), 2 = the graded panels of one of
 * its near edges exceeded the kernel's capacity (the deepest panels were dropped), 4 = a
 * weight of the pair is NaN or Inf.  `workspace` of at least rrq_workspace_size bytes.
 * The inputs are checked on the device first (as in rrq_pair_offsets, and pair_off against
 * the near list and out_len); if the check fails the call's kernels write nothing.  If
 * `stats` (HOST) is non-NULL the call synchronises the stream, fills it, and returns
 * RRQ_ERR_ARG (near list, self indices or targets invalid), RRQ_ERR_BUFFER (pair offsets
 * inconsistent or beyond out_len) or RRQ_ERR_NONFINITE (NaN or Inf weights written);
 * without stats those conditions are not reported by this call. */
rrq_status rrq_assemble(const rrq_plan* plan, const rrq_targets* tg, uint32_t kmask,
                        uint32_t flags, double* out_S, double* out_D, double* out_Sp,
                        double* out_Dp, int64_t out_len, const int64_t* pair_off,
                        uint32_t* pair_flags, void* workspace, size_t workspace_bytes,
                        void* stream, rrq_stats* stats);

/* Allocation-free variant of rrq_assemble, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation and the same output, with the workspace taken from a device array inside
 * the library, RRQ_NOALLOC_SCRATCH_BYTES (64 MiB) per GPU, held from the first call on that
 * GPU until the process ends.  Near lists whose rrq_workspace_size exceeds that return
 * RRQ_ERR_BUFFER before any launch (about 46,000 pairs when the largest order is 8).  The call
 * issues no hipMalloc, hipFree or memset, takes no statistics, and needs pair_off from
 * rrq_pair_offsets; out_len and pair_flags as for rrq_assemble.  All calls on one GPU share that GPU's array: calls that overlap in time
 * on one GPU (other streams, other threads) race and must be serialised by the caller. */
#define RRQ_NOALLOC_SCRATCH_BYTES (64ll << 20)
rrq_status rrq_assemble_noalloc(const rrq_plan* plan, const rrq_targets* tg, uint32_t kmask,
                                uint32_t flags, double* out_S, double* out_D, double* out_Sp,
                                double* out_Dp, int64_t out_len, const int64_t* pair_off,
                                uint32_t* pair_flags, void* stream);

/* pot[t] = sum over the near pairs of target t of W[block] . density[nodes of P]
 * (the sparse correction applied to nodal densities).  pot_* are [T]. */
rrq_status rrq_apply(const rrq_plan* plan, const rrq_targets* tg, uint32_t kmask,
                     const double* w_S, const double* w_D, const double* w_Sp,
                     const double* w_Dp, const int64_t* pair_off, const double* density,
                     double* pot_S, double* pot_D, double* pot_Sp, double* pot_Dp,
                     void* stream);

/* Potentials mode (the correction applied on the fly, without storing weights): pot_K[t] =
 * sum over the near pairs (t, P) of W_K[t, P] . density[nodes of P], the same numbers that
 * rrq_assemble followed by rrq_apply gives, up to rounding order.  Each pair's row of
 * integrals (the output of the translation, Sec. 3.4-3.7) is contracted with the patch
 * coefficients c_K = M_K density_P (Sec. 3.2: the fit applied to the density once per
 * patch) instead of with M_K itself, so the work per pair drops from a row-by-matrix
 * product to a dot product; with RRQ_F_CORRECTION the smooth rule over the patch nodes
 * (self node excluded) is subtracted per pair.  density is [N] (device, the surface's node
 * order); pot_* are [T] device arrays (NULL for a kernel not in kmask).  Batched form only
 * (RRQ_F_PLAIN -> RRQ_ERR_UNSUPPORTED); RRQ_F_LEARNED needs an installed network.  Uses the
 * rrq_assemble workspace; needs no pair offsets.  pair_flags (bit 4: a NaN or Inf pair
 * potential) and `stats` as for rrq_assemble. */
rrq_status rrq_potentials(const rrq_plan* plan, const rrq_targets* tg, uint32_t kmask,
                          uint32_t flags, const double* density, double* pot_S, double* pot_D,
                          double* pot_Sp, double* pot_Dp, uint32_t* pair_flags,
                          void* workspace, size_t workspace_bytes, void* stream,
                          rrq_stats* stats);

/* The smooth quadrature rule summed directly over every surface node (the self node of an
 * on-surface target excluded): pot_K[t] = sum_j w_j K(x_t, y_j) density[j] (the far-field
 * rule of Sec. 4; O(T N) work, meant for small meshes and end-to-end checks, where a fast
 * summation method would serve a large one).  Adding rrq_potentials with RRQ_F_CORRECTION
 * gives the layer potentials at the targets.  Asynchronous. */
rrq_status rrq_smooth_potentials(const rrq_plan* plan, const rrq_targets* tg, uint32_t kmask,
                                 const double* density, double* pot_S, double* pot_D,
                                 double* pot_Sp, double* pot_Dp, void* stream);

/* Autotuner of the batched form: runs the assembly of this near list for every tile size
 * (targets per workgroup: 4, 8, where the order's LDS allows it) and grid size (512, 1024,
 * 2048, 4096 persistent workgroups), times every order's tile kernel with HIP events on
 * `stream`, and keeps for each patch order its own fastest (tile, grid) in the plan.  If
 * `cache_path` (HOST, may be NULL) names a readable file written by an earlier call with the
 * same patch orders and counts, its choices are loaded instead of timing; otherwise they are
 * written there.  Synchronous.  Overwrites the output buffers.  Index i of the per-order
 * arrays is order 4, 5, 6, 8, 10 for i = 0..4 (0 for absent orders). */
typedef struct {
  int32_t tile_targets;   /* choice of the order with the longest tuned kernel time          */
  int32_t grid;
  double best_ms;         /* sum over orders of the tuned kernel times                       */
  int32_t from_cache;
  int32_t order_tile[5];
  int32_t order_grid[5];
  double order_ms[5];
} rrq_tune_result;
rrq_status rrq_autotune(rrq_plan* plan, const rrq_targets* tg, uint32_t kmask, uint32_t flags,
                        double* out_S, double* out_D, double* out_Sp, double* out_Dp,
                        int64_t out_len, const int64_t* pair_off, void* workspace,
                        size_t workspace_bytes, const char* cache_path, void* stream,
                        rrq_tune_result* result);

/* One whole assembly step (rrq_plan_refit, rrq_pair_offsets, rrq_assemble with the given
 * arguments) captured into a HIP graph; rrq_graph_launch replays it on `stream`.  In the
 * graph the fits (the maps, needed only by the tile kernels) run on a branch of their own
 * beside the edge tables, pair offsets, binning and pre-passes, joined before the tile
 * kernels.  The
 * graph holds the pointers it was created with: the buffers must stay allocated and the
 * sizes unchanged until rrq_graph_destroy; their contents (surface, targets) may change
 * between replays.  Nothing in the captured step allocates memory or issues memset/memcpy
 * nodes.  With patches of several orders the orders' tile kernels are branches of the graph
 * that run side by side.  rrq_graph_create first runs the step once, eagerly, on a stream of
 * its own that waits for the work already queued on `stream` (the caller's), then captures
 * it; it returns when that pass has finished. */
typedef struct rrq_graph rrq_graph;
rrq_status rrq_graph_create(rrq_plan* plan, const rrq_surface* surf, const rrq_targets* tg,
                            uint32_t kmask, uint32_t flags, double* out_S, double* out_D,
                            double* out_Sp, double* out_Dp, int64_t out_len, int64_t* pair_off,
                            void* workspace, size_t workspace_bytes, void* stream,
                            rrq_graph** out);
rrq_status rrq_graph_launch(rrq_graph* g, void* stream);
rrq_status rrq_graph_destroy(rrq_graph* g);

/* ---------------------------------------------------------------------------------------
 * Learned initial guess of the singularity-swap Newton solve.  The paper finds the complex
 * root t0 of sum_c (r_c(t) - x_c)^2 (eq. complexparameter) by Newton from the chord start
 * (Sec. 3.5, Step 5); it has no learned part.  Here a network 8 -> 64 -> 64 -> 2 (tanh
 * hidden units, float32) predicts dt = t0 - t_s from features of the edge and the target:
 * t_s (2), and the quadratic and cubic Legendre coefficients of the edge over the chord
 * half-length, in the chord frame (6).  With RRQ_F_LEARNED the batched form starts Newton
 * at t_s + dt and accepts the root if Newton converges within 8 iterations to a root inside
 * the Bernstein ellipse of radius rho_far; otherwise plain Newton from t_s decides.
 * Parameter vector (float32, RRQ_MLP_PARAMS): W1 [64][8], b1 [64], W2 [64][64], b2 [64],
 * W3 [2][64], b3 [2], row-major, in this order.
 * --------------------------------------------------------------------------------------- */
#define RRQ_MLP_PARAMS 4866

typedef struct {
  int32_t steps;   /* Adam steps                                                        */
  int32_t batch;   /* samples per step (drawn with replacement), 1 .. 65536              */
  float lr;        /* peak learning rate (cosine decay to 5 % of it)                     */
  uint32_t seed;   /* seeds the initial weights and the sample draws                     */
} rrq_mlp_cfg;

/* Training samples produced by the method itself: for every near pair and edge whose chord
 * start lies inside the Bernstein ellipse of radius rho_far and whose plain Newton solve
 * converges to a root inside it, in pair order: feat [8][cap] (float32, SoA), dt [2][cap]
 * (float32, t0 - t_s) and t0 [2][cap] (float64, may be NULL).  *count (HOST) = samples
 * written (at most cap).  Synchronous; allocates and frees temporary device memory. */
rrq_status rrq_collect_roots(const rrq_plan* plan, const rrq_targets* tg, int64_t cap,
                             float* feat, float* dt, double* t0, int64_t* count, void* stream);

/* Train the network on m samples (feat [8][m], dt [2][m], device) with the library's own
 * forward, backward and Adam kernels (inputs and targets are standardised during training;
 * the standardisation is folded into the returned parameters).  params [RRQ_MLP_PARAMS]
 * (device) receives the result, loss_curve [steps] (device, may be NULL) the mean squared
 * error of every step in standardised units.  Deterministic for a given seed.
 * Synchronous; allocates and frees temporary device memory. */
rrq_status rrq_mlp_train(const float* feat, const float* dt, int64_t m, const rrq_mlp_cfg* cfg,
                         float* params, float* loss_curve, void* stream);

/* Mean squared error L = (1/n) sum_b sum_o (y_bo - dt_ob)^2 of the network `params` on n
 * samples (1 <= n <= 65536) and its gradient with respect to the parameters, with the same
 * kernels as the training (gradient check).  loss [1], grad [RRQ_MLP_PARAMS] device.
 * Synchronous; allocates and frees temporary device memory. */
rrq_status rrq_mlp_loss_grad(const float* params, const float* feat, const float* dt, int64_t n,
                             float* loss, float* grad, void* stream);

/* Network outputs out [2][n] for features feat [8][n] (device).  Asynchronous. */
rrq_status rrq_mlp_predict(const float* params, const float* feat, int64_t n, float* out,
                           void* stream);

/* Give the plan a trained parameter vector (device, copied on `stream`; NULL removes it).
 * RRQ_F_LEARNED needs one (else RRQ_ERR_ARG); it is not supported with RRQ_F_PLAIN. */
rrq_status rrq_plan_set_mlp(rrq_plan* plan, const float* params, void* stream);

const char* rrq_status_string(rrq_status s);

#ifdef __cplusplus
}
#endif
#endif /* RRQ_H */
