// Internal declarations shared by the host runtime and the kernels of the RRQ library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/rrq.h"
#include "rrq_consts.h"

namespace rrq {

// constant tables of one order, on the device
struct OrderDev {
  int q, pt, np, njk;
  const double* gl_t;
  const double* gl_w;
  const double* glq_w;
  const double* LT;         // Legendre transform of GL samples
  const double* DP;         // Legendre derivatives at the GL nodes
  const double* lag_m1;
  const double* bary;       // barycentric weights of the ptilde GL nodes
  const double* bary1;      // first-form weights 1 / prod_{j != i} (t_i - t_j)
  const int32_t* dlp_ptr;
  const Term* dlp;
  const int32_t* slp_ptr;
  const Term* slp;
  const int32_t* mrg_ptr;
  const Term2* mrg;
  const int32_t* tslot;     // translation work slots (see OrderTables::tslot)
  int nslot;
  const int32_t* tlen;      // terms per slot
  const int4* tnr;          // [tchunks + 1][nslot]: 4 steps of vq_rec(n) << 8 | r (see OrderTables)
  const double4* tcf;       // [4 tchunks][nslot]: cDr, cDi, cSr, cSi (step-major)
};

// per-patch data layout constants
__host__ __device__ constexpr int64_t map_doubles(int q) { return 13LL * np_of(q) * q * q; }
__host__ __device__ constexpr int64_t tab_doubles(int q) { return 4LL * njk_of(q) * (2 * q) * 12; }
constexpr int kFrame = 16;   // o[3], ex[3], ey[3], ez[3], s, pad

struct PlanDev {
  int32_t npatch;
  int64_t N, E;
  const int32_t* order;
  const int64_t* node_off;
  const int64_t* edge_off;
  const double* node_xyz;   // [3][N] plan copy (global coordinates)
  const double* node_nrm;
  const double* node_wt;
  double* frame;            // [P][kFrame]
  double* node_loc;         // [6][N] local coordinates and normals
  double* edge_loc;         // [3][E]
  double* edge_tan;         // [3][E]
  double* edge_coef;        // [3][E] Legendre coefficients per edge
  double* edge_chord;       // [P][4][6]: chord midpoint m and half-vector d of each edge
  double* maps;             // per patch: M_D [4np][q^2], M_Sp [4np][q^2], M_S [5np][q^2]
  const int64_t* map_off;
  double* tabs;             // per patch: [4 pt][6][njk] (re, im): c (3 cplx), h (3 cplx)
  const int64_t* tab_off;
  const float* mlp;         // learned-guess network, ABI parameter layout (or null)
  double* fitcond;          // [P][2]: ||A_w||_F ||A_w^+||_F of the DLP and SLP fits
};

struct TargetsDev {
  int64_t T, nnz;
  const double* xyz;
  const double* nrm;
  const int32_t* self_patch;
  const int32_t* self_node;
  const int64_t* near_ptr;
  const int32_t* near_patch;
  // validation word of the call (in its workspace), or null: non-zero when the near list,
  // the self indices or the pair offsets failed the device check (kBad* bits); every kernel
  // that indexes with them then returns at once
  const unsigned* bad;
};
enum : unsigned { kBadNear = 1u, kBadSelf = 2u, kBadOffsets = 4u, kBadTarget = 8u };
__device__ __forceinline__ bool input_bad(const TargetsDev& tg) {
  return tg.bad != nullptr && *(const volatile unsigned*)tg.bad != 0u;
}

// statistics counters of a call (workspace): indices
enum {
  kCNear = 0,        // (pair, edge) slots integrated by singularity swap
  kCIters = 1,       // Newton iterations
  kCFail = 2,        // Newton solves that did not converge (plain rule used)
  kCLearn = 3,       // learned starts accepted
  kCMax = 4,         // largest iteration count of one slot
  kCNearList = 5,    // length of the near-slot list (root pre-pass -> near-edge moments)
  kCOverflow = 6,    // near slots whose graded panels exceeded the capacity
  kCNonfinite = 7,   // non-finite outputs (weights or pair potentials)
  kCFlagged = 8,     // pairs with a non-zero flag word
  kCWaveIters = 9,   // sum over wavefronts of the largest Newton iteration count of a lane
  kCNewtonSlots = 10,  // slots that ran Newton
  kCNewtonOver = 11,   // [5]: of those, the ones that took more than kNewtonOver[i] iterations
  kCQueueList = 16,    // length of the Newton list (slots whose chord root needs Newton)
  kCRetryList = 17,    // length of the retry list (learned starts rejected)
  kNumCounters = 18
};
constexpr int kNewtonOver[5] = {2, 4, 6, 8, 12};
// per-pair flag bits (rrq_assemble's pair_flags)
enum : uint32_t { kFlagNewton = 1u, kFlagPanels = 2u, kFlagNonfinite = 4u };
__device__ __forceinline__ void flag_pair(uint32_t* pf, unsigned long long* counters, int64_t k,
                                          uint32_t bit) {
  if (pf == nullptr) return;
  if (atomicOr(pf + k, bit) == 0u) atomicAdd(&counters[kCFlagged], 1ull);
}

struct AssembleOut {
  double* w[4];      // S, D, Sp, Dp
  uint32_t kmask, flags;
  const int64_t* pair_off;
  const int64_t* owner;     // [nnz] target of each pair
  unsigned long long* counters;   // [kNumCounters] stats
  uint32_t* pflags;         // [nnz] per-pair flag words (kFlag* bits)
  const double2* root;      // [4 nnz] singularity-swap roots t0 (root pre-pass)
  const uint8_t* nearf;     // [4 nnz] 1: singularity-swap class, 0: plain rule
  const double* lamg;       // [4 nnz][lam_stride] near-edge moments (near slots only)
  int lam_stride;
  // per pair at its position in patch order (the binning's permutation), the tile kernel's
  // target data: ptd[16 i ..] = target and its normal in the patch frame, u, global point,
  // global normal, self node (or -1); pti[4 i ..] = pair k, target, output offset, 0
  const double* ptd;
  const int64_t* pti;
  // potentials mode
  const double* dens;       // [N] nodal density
  const double* pcoef;      // [P][kCoefStride] c_D, c_S', c_S of every patch
  double* pairpot;          // [nnz][4] potential of every pair
};
constexpr int kCoefStride = 13 * np_of(kMaxQ);

struct SolveOpts {
  double rho_far, newton_tol;
  int newton_maxit;
};

// launchers (return hipError_t of the launch)
hipError_t launch_geometry(const PlanDev& pd, const rrq_surface& s, const OrderDev& od,
                           const int32_t* patches, int count, hipStream_t st);
hipError_t launch_edge_tables(const PlanDev& pd, const OrderDev& od, const int32_t* patches,
                              int count, hipStream_t st);
hipError_t launch_fit(const PlanDev& pd, const OrderDev& od, const int32_t* patches, int count,
                      double* ws, int64_t ws_per_block, int blocks, hipStream_t st);
// device check of the near list and self indices (and, with pair_off, of the pair offsets
// against out_len) into *bad; clears *bad and the counters (if given) first
hipError_t launch_validate(const PlanDev& pd, const TargetsDev& tg, const int64_t* pair_off,
                           int64_t out_len, unsigned* bad, unsigned long long* counters,
                           hipStream_t st);
// owner[k] = target of near pair k; pflags[k] = 0 (if given)
hipError_t launch_owner(const TargetsDev& tg, int64_t* owner, uint32_t* pflags,
                        hipStream_t st);
hipError_t launch_pair_offsets(const PlanDev& pd, const TargetsDev& tg, int64_t* pair_off,
                               int64_t* part, hipStream_t st);
// inclusive scan of a[1..n] in place; part holds scan_partials(n) int64
hipError_t launch_scan_i64(int64_t* a, int64_t n, int64_t* part, hipStream_t st);
int64_t scan_partials(int64_t n);
hipError_t launch_pair_plain(int q, const PlanDev& pd, const OrderDev& od, const TargetsDev& tg,
                             const AssembleOut& out, const SolveOpts& so, hipStream_t st);
hipError_t launch_apply(const PlanDev& pd, const TargetsDev& tg, const double* const* w,
                        uint32_t kmask, const int64_t* pair_off, const int64_t* owner,
                        const double* density, double* const* pot, hipStream_t st);

// first position of each order's patches in the order-grouped patch permutation; off[n] = P
// The accelerator has 8 compute dies (XCDs), each with its own L2.  The workgroups of a launch
// are handed to the dies round-robin, so blockIdx.x % kXcds names a workgroup's die.  Each
// order's tile range is cut into kXcds contiguous chunks with one queue counter each; a
// workgroup drains its own die's chunk first, so a patch's maps and tables are fetched into
// one L2 instead of all of them.
constexpr int kXcds = 8;

struct BinOrders {
  int32_t off[kNumOrders + 1];     // first position of each order's patches in perm
  int32_t tile_of_q[kMaxQ + 1];    // targets per tile for the patches of order q
};

hipError_t launch_binning(const TargetsDev& tg, int P, const int32_t* order,
                          const int32_t* perm, const BinOrders& bo, int32_t* cnt, int32_t* fill,
                          int64_t* start, int64_t* tstart, int64_t* ntiles, int64_t* sorted,
                          int4* tiles, int64_t* qtile, unsigned long long* qctr, hipStream_t st);
hipError_t launch_pair_tile(int q, int T, bool pot, int grid, const PlanDev& pd,
                            const OrderDev& od, const TargetsDev& tg, const AssembleOut& out,
                            const SolveOpts& so, const int4* tiles, const int64_t* qtile,
                            unsigned long long* qctr, const int64_t* sorted, hipStream_t st);
hipError_t launch_patch_coef(const PlanDev& pd, const double* dens, double* pcoef, hipStream_t st);
hipError_t launch_pot_reduce(const TargetsDev& tg, uint32_t kmask, const double* pairpot,
                             double* const* pot, hipStream_t st);
hipError_t launch_smooth_direct(const PlanDev& pd, const TargetsDev& tg, uint32_t kmask,
                                const double* dens, double* const* pot, hipStream_t st);
size_t tile_lds_bytes(int q, int T);
int tile_supported(int q, int T);

int64_t fit_ws_doubles(int q);
// flags[P] = 1 if the patch's frame, local geometry, maps or edge tables hold a NaN or Inf
hipError_t launch_patch_check(const PlanDev& pd, int32_t* flags, hipStream_t st);

struct RootOpts {
  double rho_far[kMaxQ + 1];
  double newton_tol;
  int newton_maxit;
};
// qlist and rlist: 4 nnz entries each (the Newton and retry lists of the root passes)
hipError_t launch_root(const PlanDev& pd, const TargetsDev& tg, const int64_t* owner,
                       const RootOpts& ro, bool learned, double2* root, uint8_t* nearf,
                       int64_t* qlist, int64_t* rlist, int64_t* nlist,
                       unsigned long long* counters, uint32_t* pflags, hipStream_t st);
// near-edge moments of every singularity-swap slot listed by the root pre-pass (counters[5]
// of them), for the patches of order q
hipError_t launch_lambda(int q, const PlanDev& pd, const OrderDev& od, const TargetsDev& tg,
                         const int64_t* owner, const double2* root, const int64_t* nlist,
                         const double* plocal, unsigned long long* counters, uint32_t* pflags,
                         double* lamg, int lam_stride, double rho_far, hipStream_t st);
// per pair k: plocal[9k ..] = target in the patch frame (3), its normal there (3), and u of
// the solid-angle integrand (3): the target normal for a self target, else the normal of the
// patch node nearest to the target (lowest index on ties) oriented toward it; and the tile
// records ptd, pti of AssembleOut at the pair's position in patch order (pair_off may be null:
// offset 0)
hipError_t launch_pair_local(const PlanDev& pd, const TargetsDev& tg, const int64_t* owner,
                             const int64_t* sorted, const int64_t* pair_off, double* plocal,
                             double* ptd, int64_t* pti, hipStream_t st);

// learned initial guess: sample collection and training
struct CollectOpts {
  double rho_far[kMaxQ + 1];
  double newton_tol;
  int newton_maxit;
};
constexpr int kMlpMomBlocks = 256;
struct MlpScratch {
  double* part;     // [kMlpMomBlocks][20] column sums
  float* stats;     // mean[10], std[10] of features and targets
  float* p;         // parameters of the normalised problem
  float* mo;        // Adam first and second moments [2][params]
  float* g;         // gradient
  float *Xn, *H1, *H2, *dY, *dH1, *dH2, *lossb;   // per-batch buffers
};
hipError_t launch_collect(const PlanDev& pd, const TargetsDev& tg, const int64_t* owner,
                          const CollectOpts& co, int pass, int64_t* flag, int64_t cap,
                          float* feat, float* dt, double* t0, hipStream_t st);
hipError_t mlp_train_run(const float* feat, const float* dt, int64_t m, int steps, int B,
                         float lr, uint64_t seed, float* params, float* loss_curve,
                         MlpScratch& s, hipStream_t st);
hipError_t mlp_loss_grad_run(const float* params, const float* feat, const float* dt,
                             int64_t n, float* loss, float* grad, MlpScratch& s,
                             hipStream_t st);
hipError_t mlp_predict_run(const float* params, const float* feat, int64_t n, float* out,
                           hipStream_t st);
hipError_t mlp_pack_run(const float* params, float* dst, hipStream_t st);


}  // namespace rrq
