// Batched form of the target-dependent steps: near pairs are binned by source patch on the
// device, and one workgroup assembles a tile of up to T targets of one patch, so that the
// patch's edge tables and coefficient maps are read once per tile and every phase has
// (target x something) parallelism.  Same arithmetic as the plain form, reorganised.
#include "rrq_device.h"
#include "rrq_internal.h"

namespace rrq {

constexpr int BNT = 256;
// panel capacity per wave: enough for every level down to kMaxLevel at the order's rho_far
__host__ __device__ constexpr int wave_panel_cap(int q) {
  return q <= 4 ? 320 : (q <= 5 ? 224 : (q <= 6 ? 144 : 112));
}

// ---------------------------------------------------------------------------------------
// binning: count pairs per patch, scan in order-grouped patch order, scatter pair indices by
// patch, emit tiles.  Tiles of one order are contiguous, [qtile[qi], qtile[qi+1]); each
// order's kernel takes them from its own kXcds queue counters qctr[qi * kXcds + c], one per
// contiguous chunk of the range (zeroed here).
// ---------------------------------------------------------------------------------------
__global__ void k_bin_clear(int32_t* cnt, int32_t* fill, int P, unsigned long long* qctr) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < P; i += gridDim.x * blockDim.x) {
    cnt[i] = 0;
    fill[i] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x < kNumOrders * kXcds) qctr[threadIdx.x] = 0;
}

__global__ void k_bin_count(TargetsDev tg, int32_t* cnt) {
  if (input_bad(tg)) return;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < tg.nnz;
       k += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&cnt[tg.near_patch[k]], 1);
}

// exclusive scans of cnt and of ceil(cnt / tile) over patches taken in the order perm
// (patches grouped by order; tile = the targets per tile of the patch's order), one workgroup
// of kBS threads with 4 KB of LDS, so that it fits on a compute unit beside a fit workgroup
// of the captured step's other branch (a 1024-thread, 16 KB version waited for one to end)
constexpr int kBS = 256;
__global__ __launch_bounds__(kBS) void k_bin_scan(const int32_t* cnt, const int32_t* perm,
                                                  BinOrders bo, int P,
                                                  int64_t* start, int64_t* tstart,
                                                  int64_t* ntiles, int64_t* qtile) {
  __shared__ int64_t s1[kBS], s2[kBS];
  __shared__ int64_t c1, c2;
  if (threadIdx.x == 0) { c1 = 0; c2 = 0; }
  __syncthreads();
  for (int base = 0; base < P; base += kBS) {
    const int i = base + threadIdx.x;
    const int pp = i < P ? perm[i] : 0;
    int tile = 1;
    for (int qi = 0; qi < kNumOrders; ++qi)
      if (i >= bo.off[qi] && i < bo.off[qi + 1]) tile = bo.tile_of_q[kOrders[qi]];
    const int64_t a = i < P ? cnt[pp] : 0;
    const int64_t b = i < P ? (cnt[pp] + tile - 1) / tile : 0;
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int o = 1; o < kBS; o <<= 1) {
      const int64_t x = threadIdx.x >= o ? s1[threadIdx.x - o] : 0;
      const int64_t y = threadIdx.x >= o ? s2[threadIdx.x - o] : 0;
      __syncthreads();
      s1[threadIdx.x] += x;
      s2[threadIdx.x] += y;
      __syncthreads();
    }
    if (i < P) {
      start[pp] = c1 + s1[threadIdx.x] - a;
      tstart[pp] = c2 + s2[threadIdx.x] - b;
      for (int qi = 0; qi < kNumOrders; ++qi)
        if (bo.off[qi] == i) qtile[qi] = c2 + s2[threadIdx.x] - b;
    }
    __syncthreads();
    if (threadIdx.x == kBS - 1) { c1 += s1[kBS - 1]; c2 += s2[kBS - 1]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *ntiles = c2;
    for (int qi = 0; qi <= kNumOrders; ++qi)
      if (bo.off[qi] >= P) qtile[qi] = c2;
  }
}

__global__ void k_bin_scatter(TargetsDev tg, const int64_t* start, int32_t* fill,
                              int64_t* sorted) {
  if (input_bad(tg)) return;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < tg.nnz;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int P = tg.near_patch[k];
    const int pos = atomicAdd(&fill[P], 1);
    sorted[start[P] + pos] = k;
  }
}

__global__ void k_bin_tiles(const int32_t* cnt, int P, const int32_t* order, BinOrders bo,
                            const int64_t* start, const int64_t* tstart, int4* tiles) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
    const int tile = bo.tile_of_q[order[p]];
    const int c = cnt[p];
    const int nt = (c + tile - 1) / tile;
    for (int j = 0; j < nt; ++j) {
      int4 v;
      v.x = p;
      v.y = (int)(start[p] + (int64_t)j * tile);   // fits in int for nnz < 2^31
      v.z = min(tile, c - j * tile);
      v.w = 0;
      tiles[tstart[p] + j] = v;
    }
  }
}

hipError_t launch_binning(const TargetsDev& tg, int P, const int32_t* order,
                          const int32_t* perm, const BinOrders& bo, int32_t* cnt, int32_t* fill,
                          int64_t* start, int64_t* tstart, int64_t* ntiles, int64_t* sorted,
                          int4* tiles, int64_t* qtile, unsigned long long* qctr, hipStream_t st) {
  const int gp = (P + 255) / 256;
  int64_t gk = (tg.nnz + 255) / 256;
  if (gk < 1) gk = 1;
  const unsigned gkk = (unsigned)(gk < 65535 ? gk : 65535);
  hipLaunchKernelGGL(k_bin_clear, dim3(gp), dim3(256), 0, st, cnt, fill, P, qctr);
  hipLaunchKernelGGL(k_bin_count, dim3(gkk), dim3(256), 0, st, tg, cnt);
  hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(kBS), 0, st, cnt, perm, bo, P, start, tstart,
                     ntiles, qtile);
  hipLaunchKernelGGL(k_bin_scatter, dim3(gkk), dim3(256), 0, st, tg, start, fill, sorted);
  hipLaunchKernelGGL(k_bin_tiles, dim3(gp), dim3(256), 0, st, cnt, P, order, bo, start, tstart,
                     tiles);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// wave-collective helpers
// ---------------------------------------------------------------------------------------

// Real-parameter Legendre series sum_k coef[3k + c] P_k(t) and its derivative, c = 0..2.
__device__ __forceinline__ void leg3r(const double* coef, int n, double t, double* r, double* dr) {
  double p0 = 0.0, p1 = 1.0, d0 = 0.0, d1 = 0.0;
  for (int c = 0; c < 3; ++c) {
    r[c] = coef[c];
    dr[c] = 0.0;
  }
  for (int k = 0; k < n - 1; ++k) {
    const double p2 = ((2.0 * k + 1.0) * t * p1 - (double)k * p0) * (1.0 / (k + 1));
    const double d2 = d0 + (2.0 * k + 1.0) * p1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    for (int c = 0; c < 3; ++c) {
      const double ck = coef[(k + 1) * 3 + c];
      r[c] += ck * p1;
      dr[c] += ck * d1;
    }
  }
}

// An opaque copy of a value: the compiler must assume it changed.  The tile kernel uses it
// so that per-lane addresses are recomputed in each phase instead of being kept live (and
// spilled) from the start of the tile.
template <typename V>
__device__ __forceinline__ V fresh(V v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Sum over the 64 lanes of x[v], v = 0..15, returned in lane l for v = (l >> 2) & 15
// (a reduce-scatter: 17 exchanges instead of 16 full reductions).  x is overwritten.
__device__ __forceinline__ double reduce_scatter16(double* x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int w = 8 >> s, o = 32 >> s;
    const bool hi = lane & o;
#pragma unroll
    for (int j = 0; j < w; ++j) {
      // selects between two values: the opaque copies keep the compiler from turning
      // them into one load at a lane-dependent index of x[] (a select chain over the
      // whole array)
      const double lo_v = fresh(x[j]), hi_v = fresh(x[w + j]);
      const double send = hi ? lo_v : hi_v;
      const double keep = hi ? hi_v : lo_v;
      x[j] = keep + __shfl_xor(send, o, 64);
    }
  }
  double v = x[0];
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 1, 64);
  return v;
}

constexpr int kMaxLevel = 52;

// Dyadic panels of [-1, 1] graded toward t0 = a + i b: a panel of half-width h and centre c
// is split while (t0 - c) / h lies inside the Bernstein ellipse of radius rho (that is,
// while its Bernstein radius is below rho).  A child's ellipse lies inside its parent's, so
// the split panels of level L form one index range [s_L, e_L], computed by lane L in closed
// form; the leaves of level L are the children of level L-1's range outside [s_L, e_L].
// Writes the leaves (lo, hi) to wpan (capacity cap) and returns their count; *over is set
// when panels were dropped.  Wave-collective.
__device__ int wave_graded_panels(double a, double b, double rho, double* wpan, int cap,
                                  bool* over) {
  const int lane = threadIdx.x & 63;
  const double A = 0.5 * (rho + 1.0 / rho), B = 0.5 * (rho - 1.0 / rho);
  const int L = lane;
  int64_t s = 0, e = -1;
  double h = ldexp(1.0, -L);
  if (L < kMaxLevel) {
    const double y = b / h;
    if (y < B) {
      const double X = A * sqrt(fmax(0.0, 1.0 - (y / B) * (y / B)));
      const double lo = (a + 1.0 - h * X) / (2.0 * h) - 0.5;
      const double hi = (a + 1.0 + h * X) / (2.0 * h) - 0.5;
      const double js = fmax(floor(lo) + 1.0, 0.0);
      const double je = fmin(ceil(hi) - 1.0, ldexp(1.0, L) - 1.0);
      if (js <= je) { s = (int64_t)js; e = (int64_t)je; }
    }
  }
  // levels are alive up to the first one with no split
  const unsigned long long split = __ballot(s <= e);
  const int lz = __builtin_ctzll(~split);        // first level with no split (< kMaxLevel)
  const int64_t ps = __shfl(s, lane > 0 ? lane - 1 : 0, 64);
  const int64_t pe = __shfl(e, lane > 0 ? lane - 1 : 0, 64);
  int64_t l0 = 0, l1 = -1, r0 = 0, r1 = -1;      // leaf index ranges of this level
  if (L == 0) {
    if (lz == 0) { l0 = 0; l1 = 0; }
  } else if (L <= lz) {
    const int64_t c0 = 2 * ps, c1 = 2 * pe + 1;   // children of level L-1's split range
    if (L == lz) { l0 = c0; l1 = c1; }
    else {
      const int64_t ss = s > c0 ? s : c0, ee = e < c1 ? e : c1;
      if (ss <= ee) {
        l0 = c0; l1 = ss - 1;
        r0 = ee + 1; r1 = c1;
      } else {
        l0 = c0; l1 = c1;
      }
    }
  }
  const int cnt = (int)((l1 - l0 + 1) + (r1 - r0 + 1));
  int incl = cnt;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o, 64);
    if (lane >= o) incl += v;
  }
  const int total = __shfl(incl, 63, 64);
  int pos = incl - cnt;
  const double w = 2.0 * h;
  for (int64_t j = l0; j <= l1; ++j, ++pos)
    if (pos < cap) { wpan[2 * pos] = -1.0 + w * (double)j; wpan[2 * pos + 1] = -1.0 + w * (double)(j + 1); }
  for (int64_t j = r0; j <= r1; ++j, ++pos)
    if (pos < cap) { wpan[2 * pos] = -1.0 + w * (double)j; wpan[2 * pos + 1] = -1.0 + w * (double)(j + 1); }
  *over = total > cap;
  return total < cap ? total : cap;
}

// ---------------------------------------------------------------------------------------
// Step 5 for every (pair, edge) slot: chord root t_s; if it lies inside the Bernstein ellipse
// of radius rho_far, Newton on the distance function.  With a network (learned form) Newton
// first starts from t_s + dt(features) for at most kLearnedMaxit iterations and keeps that
// root if it converges inside the ellipse; otherwise plain Newton from t_s decides.
// root[slot] = t0 (Im t0 >= 0), nearf[slot] = 1 for the singularity-swap class.
//
// Three passes, each over a list packed across the whole grid, so that every wavefront of a
// Newton pass is full and a lane's iteration count competes only with slots of the same
// pass: classification (chord root of every slot; Newton list), Newton from the chord start
// or from the learned start (near list; learned form: retry list of the rejected guesses),
// and, in the learned form, plain Newton over the retry list.  List entries are reserved
// once per 1024-slot chunk (classification) or per wavefront (Newton passes).  Counters: near edges, iterations, failures, learned accepts, largest
// count, the sum over wavefronts of their largest count, and the count histogram.
// ---------------------------------------------------------------------------------------
constexpr int kLearnedMaxit = 8;
constexpr int kItsShift = 56;            // retry entries: learned iterations above the slot

// Geometry of a slot: pair k, order q, target in the patch frame, edge coefficients
// (component-major, read in place).
struct RootSlot {
  int64_t k;
  int q, PT;
  double xl[3];
  const double* cf;
  const double* chord;      // m[3], d[3]
};

__device__ __forceinline__ RootSlot root_slot(const PlanDev& pd, const TargetsDev& tg,
                                              const int64_t* owner, int64_t slot) {
  RootSlot r;
  r.k = slot >> 2;
  const int e = (int)(slot & 3);
  const int P = tg.near_patch[r.k];
  r.q = pd.order[P];
  r.PT = 2 * r.q;
  const int64_t g = owner[r.k];
  const double xg[3] = {tg.xyz[g], tg.xyz[tg.T + g], tg.xyz[2 * tg.T + g]};
  frame_point(pd.frame + (int64_t)P * kFrame, xg, r.xl);
  r.cf = pd.edge_coef + pd.edge_off[P] + (int64_t)e * r.PT;
  r.chord = pd.edge_chord + ((int64_t)P * 4 + e) * 6;
  return r;
}

// Appends v of the lanes with take set to list, one counter reservation per wavefront;
// called by every lane of the wavefront.
__device__ __forceinline__ void wave_append(bool take, int64_t v, int64_t* list,
                                            unsigned long long* ctr) {
  const unsigned long long m = __ballot(take);
  if (m == 0ull) return;
  const int lane = threadIdx.x & 63, lead = __builtin_ctzll(m);
  long long b = 0;
  if (lane == lead) b = (long long)atomicAdd(ctr, (unsigned long long)__popcll(m));
  b = __shfl(b, lead, 64);
  if (take) list[b + __popcll(m & ((1ull << lane) - 1ull))] = v;
}

// Per-thread statistics of the Newton slots, folded into the counters at the kernel's end.
struct RootCounts {
  unsigned long long near = 0, iters = 0, fail = 0, learn = 0, most = 0, wave = 0, slots = 0;
  unsigned long long over[5] = {0, 0, 0, 0, 0};
  __device__ __forceinline__ void finish(int its) {
    iters += (unsigned long long)its;
    if ((unsigned long long)its > most) most = its;
    ++slots;
#pragma unroll
    for (int j = 0; j < 5; ++j) over[j] += its > kNewtonOver[j];
  }
  // a wavefront takes as long as its slowest lane: the largest count of the round
  __device__ __forceinline__ void wave_max(int its_lane) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) its_lane = max(its_lane, __shfl_xor(its_lane, o, 64));
    if ((threadIdx.x & 63) == 0) wave += (unsigned long long)its_lane;
  }
  __device__ void fold(unsigned long long* counters) {
    __shared__ unsigned long long cs[12];
    const int tid = threadIdx.x;
    if (tid < 12) cs[tid] = 0;
    __syncthreads();
    if (near) atomicAdd(&cs[0], near);
    if (iters) atomicAdd(&cs[1], iters);
    if (fail) atomicAdd(&cs[2], fail);
    if (learn) atomicAdd(&cs[3], learn);
    if (most) atomicMax(&cs[4], most);
    if (wave) atomicAdd(&cs[5], wave);
    if (slots) atomicAdd(&cs[6], slots);
#pragma unroll
    for (int j = 0; j < 5; ++j)
      if (over[j]) atomicAdd(&cs[7 + j], over[j]);
    __syncthreads();
    if (tid < 12 && cs[tid]) {
      if (tid == 4) atomicMax(&counters[kCMax], cs[4]);
      else if (tid < 4) atomicAdd(&counters[tid], cs[tid]);
      else if (tid == 5) atomicAdd(&counters[kCWaveIters], cs[5]);
      else atomicAdd(&counters[kCNewtonSlots + (tid - 6)], cs[tid]);
    }
  }
};

__global__ __launch_bounds__(256) void k_root_classify(PlanDev pd, TargetsDev tg,
                                                       const int64_t* owner, RootOpts ro,
                                                       double2* root, uint8_t* nearf,
                                                       int64_t* qlist,
                                                       unsigned long long* counters) {
  // chunks of kC slots per workgroup: the chunk's Newton slots are gathered in LDS and the
  // list is reserved once per chunk (one counter atomic per kC slots, not per wavefront)
  constexpr int kC = 1024;
  __shared__ int16_t qs[kC];   // offsets in the chunk (2 KB: shares a CU with a fit workgroup)
  __shared__ int qn;
  __shared__ long long qbase;
  if (input_bad(tg)) return;
  const int tid = threadIdx.x;
  const int64_t nslot = 4 * tg.nnz;
  for (int64_t base = (int64_t)blockIdx.x * kC; base < nslot; base += (int64_t)gridDim.x * kC) {
    __syncthreads();
    if (tid == 0) qn = 0;
    __syncthreads();
    for (int i = tid; i < kC; i += blockDim.x) {
      const int64_t slot = base + i;
      if (slot >= nslot) break;
      const RootSlot r = root_slot(pd, tg, owner, slot);
      const cplx ts = chord_root(r.chord, r.chord + 3, r.xl);
      if (bernstein_rho(ts) <= ro.rho_far[r.q]) {
        qs[atomicAdd(&qn, 1)] = (int16_t)i;
      } else {
        root[slot] = make_double2(ts.re, ts.im);
        nearf[slot] = 0;
      }
    }
    __syncthreads();
    if (tid == 0)
      qbase = qn > 0 ? (long long)atomicAdd(&counters[kCQueueList], (unsigned long long)qn) : 0;
    __syncthreads();
    for (int i = tid; i < qn; i += blockDim.x) qlist[qbase + i] = base + qs[i];
  }
}

// MODE 0: plain Newton from the chord start over the Newton list; 1: Newton from the learned
// start over the Newton list, rejected slots to the retry list; 2: plain Newton over the retry
// list, with the learned iterations added to the slot's count.
// tanh for the learned start only: 1 - 2 / (1 + e^{2x}) with the hardware base-2 exponential
// and reciprocal (absolute error about 1e-7; the network's output only seeds Newton, whose
// converged root does not depend on it).  Saturates to +-1 for large |x|.
__device__ __forceinline__ float guess_tanh(float x) {
  const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * x);   // e^{2x} = 2^{2x log2 e}
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + e);
}

template <int MODE>
__global__ __launch_bounds__(256) void k_root_newton(PlanDev pd, TargetsDev tg,
                                                     const int64_t* owner, RootOpts ro,
                                                     double2* root, uint8_t* nearf,
                                                     const int64_t* list, int64_t* rlist,
                                                     int64_t* nlist,
                                                     unsigned long long* counters,
                                                     uint32_t* pflags,
                                                     const float* __restrict__ mw) {
  if (input_bad(tg)) return;
  constexpr int kNT = 256;
  RootCounts c;
  const int tid = threadIdx.x;
  const int64_t n = (int64_t)counters[MODE == 2 ? kCRetryList : kCQueueList];
  for (int64_t i0 = (int64_t)blockIdx.x * kNT; i0 < n; i0 += (int64_t)gridDim.x * kNT) {
    const int64_t i = i0 + tid;
    int its = 0;
    bool near = false, retry = false;
    int64_t slot = 0;
    if (i < n) {
      const int64_t ent = list[i];
      slot = MODE == 2 ? (ent & ((1ll << kItsShift) - 1)) : ent;
      const RootSlot r = root_slot(pd, tg, owner, slot);
      if (MODE == 1) {
        float x[kMlpIn];
        cplx ts;
        edge_features(r.cf, r.PT, r.xl, x, &ts, 1, pd.E);
        // Parameters in the ABI layout, read at wave-uniform addresses (scalar loads, no LDS
        // traffic); the hidden layer h1 is indexed by constants only (unrolled loops), so it
        // stays in registers, and one first-layer unit is finished (fence) before the next
        // starts, which bounds the registers the tanh evaluations take.
        float h1[kMlpH];
#pragma unroll
        for (int u = 0; u < kMlpH; ++u) {
          float a = mw[kMlpB1 + u];
#pragma unroll
          for (int cc = 0; cc < kMlpIn; ++cc) a += mw[kMlpW1 + u * kMlpIn + cc] * x[cc];
          h1[u] = guess_tanh(a);
          __builtin_amdgcn_sched_barrier(0);
        }
        float y0 = mw[kMlpB3], y1 = mw[kMlpB3 + 1];
#pragma unroll 1
        for (int u = 0; u < kMlpH; ++u) {
          float a = mw[kMlpB2 + u];
#pragma unroll
          for (int kk = 0; kk < kMlpH; ++kk) a += mw[kMlpW2 + u * kMlpH + kk] * h1[kk];
          const float h2 = guess_tanh(a);
          y0 += mw[kMlpW3 + u] * h2;
          y1 += mw[kMlpW3 + kMlpH + u] * h2;
        }
        cplx tp = mk(ts.re + (double)y0, ts.im + (double)y1);
        if (isfinite(tp.re) && isfinite(tp.im)) {
          const int conv = newton_solve(r.cf, r.PT, r.xl, &tp, ro.newton_tol, kLearnedMaxit,
                                        &its, 1, pd.E);
          if (tp.im < 0) tp.im = -tp.im;
          near = conv && bernstein_rho(tp) <= ro.rho_far[r.q];
        }
        if (near) {
          ++c.learn;
          ++c.near;
          c.finish(its);
          root[slot] = make_double2(tp.re, tp.im);
          nearf[slot] = 1;
        } else {
          retry = true;
        }
      } else {
        const int its0 = MODE == 2 ? (int)(ent >> kItsShift) : 0;
        cplx tp = chord_root(r.chord, r.chord + 3, r.xl);
        const int conv = newton_solve(r.cf, r.PT, r.xl, &tp, ro.newton_tol, ro.newton_maxit,
                                      &its, 1, pd.E);
        if (tp.im < 0) tp.im = -tp.im;
        near = conv && bernstein_rho(tp) <= ro.rho_far[r.q];
        if (!conv) {
          ++c.fail;
          flag_pair(pflags, counters, r.k, kFlagNewton);
        }
        c.near += near;
        c.finish(its0 + its);
        root[slot] = make_double2(tp.re, tp.im);
        nearf[slot] = (uint8_t)near;
      }
    }
    c.wave_max(its);
    wave_append(near, slot, nlist, &counters[kCNearList]);
    if (MODE == 1)
      wave_append(retry, slot | ((int64_t)its << kItsShift), rlist, &counters[kCRetryList]);
  }
  c.fold(counters);
}

hipError_t launch_root(const PlanDev& pd, const TargetsDev& tg, const int64_t* owner,
                       const RootOpts& ro, bool learned, double2* root, uint8_t* nearf,
                       int64_t* qlist, int64_t* rlist, int64_t* nlist,
                       unsigned long long* counters, uint32_t* pflags, hipStream_t st) {
  const int64_t nslot = 4 * tg.nnz;
  int64_t g = (nslot + 1023) / 1024;
  if (g < 1) g = 1;
  const dim3 gc((unsigned)(g < 4096 ? g : 4096)), gn(1024), b(256);
  const float* mw = (const float*)pd.mlp;
  hipLaunchKernelGGL(k_root_classify, gc, b, 0, st, pd, tg, owner, ro, root, nearf, qlist,
                     counters);
  if (learned) {
    hipLaunchKernelGGL(k_root_newton<1>, gn, b, 0, st, pd, tg, owner, ro, root, nearf, qlist,
                       rlist, nlist, counters, pflags, mw);
    hipLaunchKernelGGL(k_root_newton<2>, gn, b, 0, st, pd, tg, owner, ro, root, nearf, rlist,
                       nullptr, nlist, counters, pflags, nullptr);
  } else {
    hipLaunchKernelGGL(k_root_newton<0>, gn, b, 0, st, pd, tg, owner, ro, root, nearf, qlist,
                       nullptr, nlist, counters, pflags, nullptr);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// LDS layout of one tile (doubles, then ints)
// ---------------------------------------------------------------------------------------
// Local coordinates xl and normal nl of a target in the frame fr of a patch (q2 nodes from
// n0), and the vector u of the solid-angle integrand: the target normal for a self target,
// else the normal of the nearest node (lowest index on ties; a scan in index order keeps the
// first of equal distances) oriented toward the target.
__device__ __forceinline__ void pair_local(const PlanDev& pd, const double* fr, int64_t n0,
                                           int q2, int self, const double* xg, const double* nv,
                                           double* xl, double* nl, double* u) {
  frame_point(fr, xg, xl);
  for (int a = 0; a < 3; ++a) {
    const double* ax = fr + 3 + 3 * a;
    nl[a] = nv[0] * ax[0] + nv[1] * ax[1] + nv[2] * ax[2];
  }
  if (self >= 0) {
    for (int c = 0; c < 3; ++c) u[c] = nl[c];
    return;
  }
  // bi starts at a valid node, so that non-finite distances still select a node
  double bd = 1e300;
  int bi = 0;
  for (int i = 0; i < q2; ++i) {
    double d2 = 0;
    for (int c = 0; c < 3; ++c) {
      const double dd = xl[c] - pd.node_loc[c * pd.N + n0 + i];
      d2 += dd * dd;
    }
    if (d2 < bd) { bd = d2; bi = i; }
  }
  double dd = 0, nn[3];
  for (int c = 0; c < 3; ++c) {
    nn[c] = pd.node_loc[(3 + c) * pd.N + n0 + bi];
    dd += (xl[c] - pd.node_loc[c * pd.N + n0 + bi]) * nn[c];
  }
  const double sg = dd >= 0.0 ? 1.0 : -1.0;
  for (int c = 0; c < 3; ++c) u[c] = sg * nn[c];
}

// Per-pair pre-pass: pair_local of every (target, patch) pair into plocal[9 k ..], and the
// pair's tile record (ptd, pti) at its position i in patch order, so that a tile reads its
// targets' data from consecutive records with no dependent loads.
__global__ __launch_bounds__(256) void k_pair_local(PlanDev pd, TargetsDev tg,
                                                    const int64_t* owner, const int64_t* sorted,
                                                    const int64_t* pair_off, double* plocal,
                                                    double* ptd, int64_t* pti) {
  if (input_bad(tg)) return;
  // pairs in patch order (the binning's permutation), so that the lanes of a wavefront
  // mostly scan the nodes of one patch
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tg.nnz;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = sorted[i];
    const int P = tg.near_patch[k];
    const int64_t g = owner[k];
    const double* fr = pd.frame + (int64_t)P * kFrame;
    const int64_t n0 = pd.node_off[P];
    const int q2 = pd.order[P] * pd.order[P];
    const int self = (tg.self_patch[g] == P) ? tg.self_node[g] : -1;
    double xg[3], nv[3], xl[3], nl[3], u[3];
    for (int c = 0; c < 3; ++c) {
      xg[c] = tg.xyz[c * tg.T + g];
      nv[c] = tg.nrm[c * tg.T + g];
    }
    pair_local(pd, fr, n0, q2, self, xg, nv, xl, nl, u);
    double* o = plocal + 9 * k;
    double* r = ptd + 16 * i;
    for (int c = 0; c < 3; ++c) {
      o[c] = r[c] = xl[c];
      o[3 + c] = r[3 + c] = nl[c];
      o[6 + c] = r[6 + c] = u[c];
      r[9 + c] = xg[c];
      r[12 + c] = nv[c];
    }
    r[15] = (double)self;
    int64_t* ri = pti + 4 * i;
    ri[0] = k;
    ri[1] = g;
    ri[2] = pair_off ? pair_off[k] : 0;
    ri[3] = 0;
  }
}

hipError_t launch_pair_local(const PlanDev& pd, const TargetsDev& tg, const int64_t* owner,
                             const int64_t* sorted, const int64_t* pair_off, double* plocal,
                             double* ptd, int64_t* pti, hipStream_t st) {
  int64_t g = (tg.nnz + 255) / 256;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_pair_local, dim3((unsigned)(g < 8192 ? g : 8192)), dim3(256), 0, st, pd,
                     tg, owner, sorted, pair_off, plocal, ptd, pti);
  return hipGetLastError();
}

// Step 5 on a near edge (the singularity-swap class): the Lagrange-basis moments of the two
// kernels |tau - t0|^m / |r(tau) - x|^m, m = 1, 3, on panels graded toward t0, and the edge's
// part of the solid angle Omega_0.  One wave per near (pair, edge), lanes over the panel
// points; a workgroup of kLamWaves waves takes items i = w, w + stride, ... from the list of
// near slots the root pre-pass wrote, skipping items of other orders.  Output per slot:
// lamg[slot * stride] = lambda^(1)[PT], lambda^(3)[PT], Omega_0 part.
constexpr int kLamWaves = 4;

template <int Q>
__global__ __launch_bounds__(64 * kLamWaves) __attribute__((amdgpu_waves_per_eu(3)))
void k_lambda(PlanDev pd, OrderDev od, TargetsDev tg, const int64_t* owner, const double2* root,
              const int64_t* nlist, const double* plocal, unsigned long long* counters,
              uint32_t* pflags, double* lamg, int lam_stride, double rho_far) {
  constexpr int PT = 2 * Q;
  constexpr int NB8 = (PT + 7) / 8;
  constexpr int NPAN = wave_panel_cap(Q);
  __shared__ double cgl_t[PT], cgl_w[PT], cbary[PT];
  __shared__ double scoef[kLamWaves][PT * 3];
  __shared__ double span[kLamWaves][NPAN * 2];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid < PT) {
    cgl_t[tid] = od.gl_t[tid];
    cgl_w[tid] = od.gl_w[tid];
    cbary[tid] = od.bary1[tid];
  }
  __syncthreads();
  if (input_bad(tg)) return;
  const int64_t nitems = (int64_t)counters[kCNearList];
  unsigned long long c_over = 0;
  double* ecoef = scoef[wv];
  double* wpan = span[wv];
  for (int64_t it = (int64_t)blockIdx.x * kLamWaves + wv; it < nitems;
       it += (int64_t)gridDim.x * kLamWaves) {
    const int64_t slot = nlist[it];
    const int64_t k = slot >> 2;
    const int e = (int)(slot & 3);
    const int P = tg.near_patch[k];
    if (pd.order[P] != Q) continue;
    const int64_t e0 = pd.edge_off[P] + (int64_t)e * PT;
    for (int i = lane; i < PT * 3; i += 64)
      ecoef[i] = pd.edge_coef[(i % 3) * pd.E + e0 + i / 3];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    double xl[3], u[3];
    for (int c = 0; c < 3; ++c) {
      xl[c] = plocal[9 * k + c];
      u[c] = plocal[9 * k + 6 + c];
    }
    const double2 r0 = root[slot];
    const double a = r0.x, b = r0.y;
    bool over;
    const int npan = wave_graded_panels(a, b, rho_far, wpan, NPAN, &over);
    if (over && lane == 0) {
      ++c_over;
      flag_pair(pflags, counters, slot >> 2, kFlagPanels);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const int npts = npan * PT;
    double lacc[NB8];
#pragma unroll
    for (int bI = 0; bI < NB8; ++bI) lacc[bI] = 0.0;
    double om = 0.0;
    for (int base = 0; base < npts; base += 64) {
      const int idx = base + lane;
      double w1p = 0.0, w3p = 0.0, tau = 3.0;
      asm volatile("" ::: "memory");   // keep the node tables out of registers
      if (idx < npts) {
        const int pn = idx / PT, gg = idx % PT;
        const double lo = wpan[pn * 2], hi = wpan[pn * 2 + 1];
        const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
        tau = c + h * cgl_t[gg];
        const double K2 = (tau - a) * (tau - a) + b * b;
        const double K1 = 1.0 / sqrt(K2);
        const double hw = h * cgl_w[gg];
        w1p = hw * K1;
        w3p = w1p / K2;
        double r[3], dr[3];
        leg3r(ecoef, PT, tau, r, dr);
        om += hw * omega0_at(xl, u, r, dr);
      }
      // Lagrange basis at tau, first barycentric form l_i = ell(tau) b_i / (tau - t_i) with
      // ell(tau) = prod_j (tau - t_j) (backward stable, and no reciprocal for the
      // denominator); 1/(tau - t_i) by the hardware reciprocal and one Newton step (relative
      // error a few ulp, against a correctly rounded divide)
      double ell = 1.0;
      int hit = -1;
#pragma unroll
      for (int j = 0; j < PT; ++j) {
        const double dtj = tau - cgl_t[j];
        if (dtj == 0.0) hit = j;
        ell *= dtj;
      }
#pragma unroll
      for (int bI = 0; bI < NB8; ++bI) {
        double x[16];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          const int i = bI * 8 + v;
          double l = 0.0;
          if (i < PT) {
            if (hit >= 0) l = hit == i ? 1.0 : 0.0;
            else l = cbary[i] * rcp_nr(tau - cgl_t[i]) * ell;
          }
          x[v] = w1p * l;
          x[8 + v] = w3p * l;
        }
        lacc[bI] += reduce_scatter16(x);
      }
    }
    om = wave_sum(om);
    double* outp = lamg + slot * lam_stride;
    if ((lane & 3) == 0) {
      const int v = lane >> 2;
#pragma unroll
      for (int bI = 0; bI < NB8; ++bI) {
        const int i = bI * 8 + (v & 7);
        if (i < PT) outp[(v >> 3) * PT + i] = lacc[bI];
      }
    }
    if (lane == 0) outp[2 * PT] = om;
    __builtin_amdgcn_wave_barrier();
  }
  if (c_over) atomicAdd(&counters[kCOverflow], c_over);
}

hipError_t launch_lambda(int q, const PlanDev& pd, const OrderDev& od, const TargetsDev& tg,
                         const int64_t* owner, const double2* root, const int64_t* nlist,
                         const double* plocal, unsigned long long* counters, uint32_t* pflags,
                         double* lamg, int lam_stride, double rho_far, hipStream_t st) {
  if (tg.nnz <= 0) return hipSuccess;
  const int grid = 2048;
  switch (q) {
#define X(Q) case Q: hipLaunchKernelGGL(k_lambda<Q>, dim3(grid), dim3(64 * kLamWaves), 0, st, pd, od, tg, owner, root, nlist, plocal, counters, pflags, lamg, lam_stride, rho_far); break;
    X(4) X(5) X(6) X(8) X(10)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// n rounded up to 4 mod 8: a per-target stride of that many doubles is 8 or 24 dwords mod 32,
// so the 8-dword spans of four consecutive targets use disjoint LDS banks
__host__ __device__ constexpr int pad_banks(int n) { return n + ((4 - n) % 8 + 8) % 8; }

// A double moved between lanes by a DPP permutation of each 16-lane row (two 32-bit moves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// v = sum of v over the aligned group of N lanes (N = 8, 16 or 32), in every lane of the
// group: quad swaps (lanes i ^ 1, i ^ 2), then the mirror within 8 lanes and within 16, which
// pair each partial sum with a disjoint one; across rows by a lane exchange.
template <int N>
__device__ __forceinline__ void row_sum(double& v) {
  static_assert(N == 8 || N == 16 || N == 32, "group of 8, 16 or 32 lanes");
  v += dpp_f64<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x141>(v);   // row_half_mirror
  if constexpr (N >= 16) v += dpp_f64<0x140>(v);   // row_mirror
  if constexpr (N == 32) v += __shfl_xor(v, 16, 64);
}

template <int Q, int T>
struct TileLds {
  static constexpr int PT = 2 * Q, NP = np_of(Q), NJK = njk_of(Q), NR = tri(Q, Q) + 1;
  static constexpr int o_fr = 0;
  static constexpr int o_x = o_fr + kFrame;                // [T][3]
  static constexpr int o_nu = o_x + 3 * T;
  static constexpr int o_u = o_nu + 3 * T;
  static constexpr int o_t0 = o_u + 3 * T;                 // [T][4][2]
  static constexpr int o_om = o_t0 + 8 * T;                // [T][4]: Omega_0, Omega_vec
  static constexpr int o_dom = o_om + 4 * T;               // [T][4]
  static constexpr int o_ids = o_dom + 4 * T;              // [T][3] i64: pair, target, offset
  static constexpr int o_xg = o_ids + 3 * T;               // [T][6]: global point, normal
  // Per-target strides of the edge-point data and of the rows, padded so that the four
  // targets a wave reads at once (lanes t = 0..3 of the contraction; the target quad of the
  // MFMA operands) fall in different LDS banks: the unpadded strides are multiples of 32
  // dwords, which put all four in one bank.
  static constexpr int TDS = 4 * PT * 8 + 2;                // doubles per target of td
  static constexpr int R4 = pad_banks(4 * NP), R5 = pad_banks(5 * NP);
  static constexpr int o_td = o_xg + 6 * T;               // [T][TDS] (aliased by rows)
  static constexpr int n_td = T * TDS;
  static constexpr int n_rows = T * (3 * R4 + R5);
  static constexpr int n_scrA = n_td > n_rows ? n_td : n_rows;
  static constexpr int o_rows = o_td;                      // rD [T][R4], rSp, rS [T][R5], rDp
  // moments per (target, (j,k)): 18 values at vq_rec(n) in the target's block of VQT
  static constexpr int VQT = vq_rec(NJK);
  static constexpr int o_vq = o_td + n_scrA;               // [T][VQT]
  static constexpr int o_part = o_vq;                      // [T][4][8]: edge partial sums,
                                                           // dead before vq is written
  static constexpr int o_rt = o_vq + T * VQT;              // [T][NR] cplx
  static constexpr int o_gs = o_rt + 2 * T * NR;           // [T][NR] cplx
  static constexpr int o_cst = o_gs + 2 * T * NR;          // gl_t, gl_w [PT] each
  static constexpr int n_dbl = o_cst + 2 * PT;
  // ints
  static constexpr int i_near = 0;                         // [T][4]
  static constexpr int i_self = i_near + 4 * T;
  static constexpr int n_int = i_self + T;
  static constexpr size_t bytes = (size_t)n_dbl * 8 + (size_t)n_int * 4 + 64;
};

// Phase timers of the tile kernel, in the profiling build only (-DRRQ_PHASE_TIMERS, library
// librrq_phases.so): thread 0 reads the shader clock at the workgroup barriers that separate
// the phases and adds the differences per phase; the sums over workgroups are read with
// rrq_phase_read.  Slots: 0 targets, 1 roots and target harmonics, 2 effective weights,
// 3 contraction, 4 translation, 5 rows x maps and stores, 6 tile fetch.
#ifdef RRQ_PHASE_TIMERS
__device__ unsigned long long g_tile_phase[8];
#define RRQ_PHASE_INIT                                        \
  unsigned long long ph_[8] = {0, 0, 0, 0, 0, 0, 0, 0};       \
  unsigned long long ph_t_ = __builtin_amdgcn_s_memtime();
#define RRQ_PHASE(i)                                          \
  if (threadIdx.x == 0) {                                     \
    const unsigned long long n_ = __builtin_amdgcn_s_memtime(); \
    ph_[i] += n_ - ph_t_;                                     \
    ph_t_ = n_;                                               \
  }
#define RRQ_PHASE_FLUSH \
  if (threadIdx.x == 0) for (int i_ = 0; i_ < 8; ++i_) atomicAdd(&g_tile_phase[i_], ph_[i_]);
#else
#define RRQ_PHASE_INIT
#define RRQ_PHASE(i)
#define RRQ_PHASE_FLUSH
#endif

// Persistent workgroups take tiles of this order from a queue, so that the workgroups in
// flight work on a narrow window of consecutive tiles (tiles of one patch are consecutive)
// and the patch's maps and edge tables are served from L2.
// Register target = the workgroups per CU that the LDS allows (160 KiB per CU): three at
// order 8 with 4 targets, which outweighs the spills that 168 VGPRs cost.
template <int Q, int T, bool POT>
__global__ __launch_bounds__(BNT)
__attribute__((amdgpu_waves_per_eu(TileLds<Q, T>::bytes <= 54 * 1024 ? 3 : (TileLds<Q, T>::bytes <= 80 * 1024 ? 2 : 1))))
void k_pair_tile(PlanDev pd, OrderDev od, TargetsDev tg,
                                                   AssembleOut out, SolveOpts so,
                                                   const int4* tiles, const int64_t* qtile,
                                                   unsigned long long* qctr,
                                                   const int64_t* sorted) {
  using L = TileLds<Q, T>;
  constexpr int PT = L::PT, NP = L::NP, NJK = L::NJK, NR = L::NR, Q2 = Q * Q;
  constexpr int PTP = PT <= 8 ? 8 : (PT <= 16 ? 16 : 32);   // lanes per (target, edge)
  constexpr int NB8 = (PT + 7) / 8;                          // blocks of 8 edge nodes
  extern __shared__ double smem[];
  __shared__ long long s_ti;
  double* fr = smem + L::o_fr;
  double* sx = smem + L::o_x;
  double* snu = smem + L::o_nu;
  double* su = smem + L::o_u;
  double* st0 = smem + L::o_t0;
  double* som = smem + L::o_om;
  double* sdom = smem + L::o_dom;
  int64_t* sids = (int64_t*)(smem + L::o_ids);   // per target: pair k, target g, pair_off[k]
  double* sxg = smem + L::o_xg;                   // per target: global point and normal
  double* part = smem + L::o_part;
  double* td = smem + L::o_td;
  double* rows = smem + L::o_rows;
  double* vq = smem + L::o_vq;
  cplx* Rt = (cplx*)(smem + L::o_rt);
  cplx* gS = (cplx*)(smem + L::o_gs);
  double* cgl_t = smem + L::o_cst;
  double* cgl_w = cgl_t + PT;
  int* ints = (int*)(smem + L::n_dbl);
  int* snear = ints + L::i_near;
  int* sself = ints + L::i_self;

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (input_bad(tg)) return;
  RRQ_PHASE_INIT
  const int64_t tlo = qtile[0], thi = qtile[1];
  if (tid < PT) {
    cgl_t[tid] = od.gl_t[tid];
    cgl_w[tid] = od.gl_w[tid];
  }
  // chunk c of the order's tiles is [tlo + len c / kXcds, tlo + len (c+1) / kXcds); the
  // workgroup starts with its own die's chunk and moves on to the next one when it is empty
  // (at most kXcds empty draws per workgroup, so every workgroup leaves the loop)
  const int64_t len = thi - tlo;
  const int xcd = blockIdx.x % kXcds;
  int round = 0;
  for (;;) {
    RRQ_PHASE(5)
    __syncthreads();
    if (tid == 0) {
      long long next = -1;
      while (round < kXcds) {
        const int c = (xcd + round) % kXcds;
        const int64_t chi = tlo + len * (c + 1) / kXcds;
        const long long v = tlo + len * c / kXcds + (long long)atomicAdd(qctr + c, 1ull);
        if (v < chi) {
          next = v;
          break;
        }
        ++round;
      }
      s_ti = next;
    }
    __syncthreads();
    RRQ_PHASE(6)
    const int64_t ti = s_ti;
    if (ti < 0) break;
    const int4 tile = tiles[ti];
    const int P = tile.x;
    if (pd.order[P] != Q) continue;
    const int64_t n0 = pd.node_off[P], e0 = pd.edge_off[P];
    for (int sub = 0; sub < tile.z; sub += T) {
      const int nt = min(T, tile.z - sub);
      __syncthreads();
      RRQ_PHASE(5)
      // ---- patch frame, and the targets' data from their tile records (32 threads per
      // target, one value each): local point, normal and u; global point and normal; self
      // node; pair, target and output offset
      if (tid < kFrame) fr[tid] = pd.frame[(int64_t)P * kFrame + tid];
      for (int it = tid; it < nt * 32; it += BNT) {
        const int t = it >> 5, f = it & 31;
        if (f >= 19) continue;
        const int64_t i = tile.y + sub + t;
        if (f < 16) {
          const double v = out.ptd[16 * i + f];
          if (f < 3) sx[t * 3 + f] = v;
          else if (f < 6) snu[t * 3 + f - 3] = v;
          else if (f < 9) su[t * 3 + f - 6] = v;
          else if (f < 15) sxg[t * 6 + f - 9] = v;
          else sself[t] = (int)v;
          continue;
        }
        const int64_t v = out.pti[4 * i + f - 16];
        sids[t * 3 + f - 16] = (f == 18 && POT) ? 0 : v;
      }
      __syncthreads();
      RRQ_PHASE(0)
      // ---- Step 5 results (root pre-pass) per (target, edge); Step 4: target harmonics
      if (tid < 4 * nt) {
        const int t = tid >> 2, e = tid & 3;
        const int64_t slot = 4 * sids[t * 3] + e;
        const double2 r = out.root[slot];
        snear[t * 4 + e] = out.nearf[slot];
        st0[(t * 4 + e) * 2] = r.x;
        st0[(t * 4 + e) * 2 + 1] = r.y;
      } else if (tid >= 64 && tid < 64 + nt) {
        const int t = tid - 64;
        solid_table<Q>(sx[t * 3 + 1], sx[t * 3 + 2], sx[t * 3 + 0], Rt + t * NR);
      }
      __syncthreads();
      RRQ_PHASE(1)
      // ---- effective weights per (target, edge, node), PTP lanes per (target, edge), and
      // the Omega sums of each (target, edge) by a segmented lane reduction
      for (int idx = tid; idx < T * 4 * PTP; idx += BNT) {
        const int te = idx / PTP, i = idx % PTP;
        const int t = te >> 2, e = te & 3;
        double om0 = 0.0, ov[3] = {0, 0, 0}, dv[3] = {0, 0, 0}, dom0 = 0.0;
        const bool act = t < nt && i < PT;
        const int near = t < nt ? snear[te] : 0;
        // near edges: lambda^(1), lambda^(3) and the Omega_0 part from the near-edge pre-pass
        const double* lg = nullptr;
        if (near) lg = out.lamg + (4 * sids[t * 3] + e) * out.lam_stride;
        if (act) {
          const double* xl = sx + t * 3;
          const double* nl = snu + t * 3;
          const double a = st0[te * 2], b = st0[te * 2 + 1];
          const int64_t ei = fresh(e0) + e * PT + i;
          double d[3], rr[3], rp[3];
          for (int c = 0; c < 3; ++c) {
            rr[c] = pd.edge_loc[c * pd.E + ei];
            rp[c] = pd.edge_tan[c * pd.E + ei];
            d[c] = xl[c] - rr[c];
          }
          const double R2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
          const double R = sqrt(R2);
          double w1, w3;
          if (near) {
            const double ta = cgl_t[i] - a;
            const double q1 = sqrt(ta * ta + b * b) / R;
            w1 = lg[i] * q1;
            w3 = lg[PT + i] * q1 * q1 * q1;
          } else {
            w1 = cgl_w[i] / R;
            w3 = cgl_w[i] / (R2 * R);
            om0 = cgl_w[i] * omega0_at(xl, su + t * 3, rr, rp);
          }
          const double dn = d[0] * nl[0] + d[1] * nl[1] + d[2] * nl[2];
          double* o = td + t * L::TDS + (e * PT + i) * 8;
          o[0] = w1;
          for (int c = 0; c < 3; ++c) {
            o[1 + c] = d[c];
            o[4 + c] = w1 * nl[c] - w3 * dn * d[c];
          }
          for (int c = 0; c < 3; ++c) {
            ov[c] = -w1 * rp[c];
            dv[c] = w3 * dn * rp[c];
          }
          const double cx = rp[1] * d[2] - rp[2] * d[1];
          const double cy = rp[2] * d[0] - rp[0] * d[2];
          const double cz = rp[0] * d[1] - rp[1] * d[0];
          dom0 = -w3 * (cx * nl[0] + cy * nl[1] + cz * nl[2]);
        }
        // sums over the PTP lanes of (target, edge): DPP lane moves within rows of 16 lanes,
        // then lane exchanges across rows (PTP = 32)
        row_sum<PTP>(om0);
        row_sum<PTP>(dom0);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          row_sum<PTP>(ov[c]);
          row_sum<PTP>(dv[c]);
        }
        if (i == 0 && t < nt) {
          double* pp = part + te * 8;
          pp[0] = near ? lg[2 * PT] : om0;
          pp[1] = ov[0]; pp[2] = ov[1]; pp[3] = ov[2];
          pp[4] = dv[0]; pp[5] = dv[1]; pp[6] = dv[2]; pp[7] = dom0;
        }
      }
      __syncthreads();
      RRQ_PHASE(2)
      if (tid < nt) {
        const int t = tid;
        double o[4] = {0, 0, 0, 0}, d[4] = {0, 0, 0, 0};
        for (int e = 0; e < 4; ++e) {
          const double* pp = part + (t * 4 + e) * 8;
          o[0] += pp[0];
          o[1] += pp[1]; o[2] += pp[2]; o[3] += pp[3];
          d[1] += pp[4]; d[2] += pp[5]; d[3] += pp[6]; d[0] += pp[7];
        }
        for (int c = 0; c < 4; ++c) { som[t * 4 + c] = o[c]; sdom[t * 4 + c] = d[c]; }
      }
      __syncthreads();   // the partial sums share their LDS with the moments written next
      // ---- Step 6: contraction with the edge tables, items (j,k) x target; then the normal
      // derivatives nu'.grad S^{ab} at the targets, items (target, a, b)
      const double* tb = pd.tabs + pd.tab_off[P];
      for (int idx = tid; idx < NJK * T + nt * NR; idx += BNT) {
        if (idx >= NJK * T) {
          const int it = idx - NJK * T;
          const int t = it / NR, r = it % NR;
          int a = 0;
          while (tri(a + 1, 0) <= r) ++a;
          const int b = r - tri(a, 0);
          cplx acc = mk(0, 0);
          for (int c = 0; c < 3; ++c) acc = acc + snu[t * 3 + c] * dS(Rt + t * NR, a, b, c);
          gS[it] = acc;
          continue;
        }
        const int n = idx / T, t = idx % T;
        if (t >= nt) continue;
        double V0 = 0, V1 = 0;
        double Qr[4] = {0, 0, 0, 0}, Qi[4] = {0, 0, 0, 0};
        double Dr[4] = {0, 0, 0, 0}, Di[4] = {0, 0, 0, 0};
        // the 4 PT edge points in order (edge-major); the table entries of the next point are
        // loaded before this point's products, so that their latency overlaps them.  The
        // lanes of a wave read consecutive (j,k) of one point and component.
        constexpr int NPTS = 4 * PT;
        const double2* ob = (const double2*)tb + n;
        const double* tdb = td + t * L::TDS;
        double cur[12];
#pragma unroll
        for (int u = 0; u < 6; ++u) {
          const double2 v = ob[u * NJK];
          cur[2 * u] = v.x;
          cur[2 * u + 1] = v.y;
        }
#pragma unroll 2
        for (int p = 0; p < NPTS; ++p) {
          const double2* onx = ob + (int64_t)min(p + 1, NPTS - 1) * 6 * NJK;
          double nx[12];
#pragma unroll
          for (int u = 0; u < 6; ++u) {
            const double2 v = onx[u * NJK];
            nx[2 * u] = v.x;
            nx[2 * u + 1] = v.y;
          }
          // keeps these loads ahead of this point's products (the scheduler would otherwise
          // sink them to the end of the loop body, next to their use)
          __builtin_amdgcn_sched_barrier(0);
          {
            const double* tdp = tdb + p * 8;
            const double w1 = tdp[0];
            const double d0 = tdp[1], d1 = tdp[2], d2 = tdp[3];
            const double a0 = tdp[4], a1 = tdp[5], a2 = tdp[6];
            const double c0r = cur[0], c0i = cur[1], c1r = cur[2], c1i = cur[3], c2r = cur[4], c2i = cur[5];
            const double h0r = cur[6], h0i = cur[7], h1r = cur[8], h1i = cur[9], h2r = cur[10], h2i = cur[11];
            // every product is accumulated with its own FMA (no temporary sums)
            const double v0 = w1 * d0, v1 = w1 * d1, v2 = w1 * d2;
            V0 = fma(v0, c0r, fma(v1, c1r, fma(v2, c2r, V0)));
            V1 = fma(v0, c0i, fma(v1, c1i, fma(v2, c2i, V1)));
            Qr[0] = fma(-v0, h0r, fma(-v1, h1r, fma(-v2, h2r, Qr[0])));
            Qi[0] = fma(-v0, h0i, fma(-v1, h1i, fma(-v2, h2i, Qi[0])));
            Qr[1] = fma(v1, h2r, fma(-v2, h1r, Qr[1]));
            Qi[1] = fma(v1, h2i, fma(-v2, h1i, Qi[1]));
            Qr[2] = fma(v2, h0r, fma(-v0, h2r, Qr[2]));
            Qi[2] = fma(v2, h0i, fma(-v0, h2i, Qi[2]));
            Qr[3] = fma(v0, h1r, fma(-v1, h0r, Qr[3]));
            Qi[3] = fma(v0, h1i, fma(-v1, h0i, Qi[3]));
            Dr[0] = fma(-a0, h0r, fma(-a1, h1r, fma(-a2, h2r, Dr[0])));
            Di[0] = fma(-a0, h0i, fma(-a1, h1i, fma(-a2, h2i, Di[0])));
            Dr[1] = fma(a1, h2r, fma(-a2, h1r, Dr[1]));
            Di[1] = fma(a1, h2i, fma(-a2, h1i, Di[1]));
            Dr[2] = fma(a2, h0r, fma(-a0, h2r, Dr[2]));
            Di[2] = fma(a2, h0i, fma(-a0, h2i, Di[2]));
            Dr[3] = fma(a0, h1r, fma(-a1, h0r, Dr[3]));
            Di[3] = fma(a0, h1i, fma(-a1, h0i, Di[3]));
          }
#pragma unroll
          for (int u = 0; u < 12; ++u) cur[u] = nx[u];
        }
        double* o = vq + t * L::VQT + vq_rec(n);
        o[0] = V0; o[1] = V1;
        for (int c = 0; c < 4; ++c) {
          o[2 + 2 * c] = Qr[c]; o[3 + 2 * c] = Qi[c];
          o[10 + 2 * c] = Dr[c]; o[11 + 2 * c] = Di[c];
        }
      }
      __syncthreads();
      RRQ_PHASE(3)
      // ---- Steps 7-8: translation and rows, items (target, slot): a slot holds the term list
      // of one (l, m) or one of the 2 or 4 pieces of a long one, on adjacent lanes
      for (int idx = tid; idx < T * od.nslot; idx += BNT) {
        const int t = idx / od.nslot, slot = idx % od.nslot, code = od.tslot[slot];
        const int lm = code & 0xff, piece = (code >> 8) & 0xf, lg = code >> 12;
        const bool act = t < nt && code != kPadSlot;
        int l = 1;
        while (np_of(l) <= lm) ++l;
        const int m = lm - np_of(l - 1) + 1;
        const int tt = t < nt ? t : 0;
        const cplx* R = Rt + tt * NR;
        const cplx* G = gS + tt * NR;
        const double* VQ = vq + tt * L::VQT;
        // imaginary parts of I[alpha] (quaternion), of its normal derivative and of the
        // single-layer sum
        double Ia[4] = {0, 0, 0, 0}, dIa[4] = {0, 0, 0, 0}, sl = 0.0;
        // one pass over the (j, k) terms of this (l, m): single-layer sum (weights D_{j,l})
        // and double-layer sums (weights C_{j,l}, zero for j = 1); the signs of conjugation
        // (k < 0) and of S^{(a,b)} for b < 0 are folded into the weights
        // (the slot's terms are read in chunks of 4 steps: one int4 of operand offsets per
        // chunk, read one chunk ahead, and the chunk's coefficients, whose addresses do not
        // depend on a load, so that a chunk waits on one memory latency)
        const int nch = act ? (od.tlen[slot] + 3) >> 2 : 0;
        const int ns = od.nslot;
        int4 nr4 = od.tnr[slot];
#pragma unroll 1
        for (int ch = 0; ch < nch; ++ch) {
          const int4 nr4n = od.tnr[(ch + 1) * ns + slot];
          const double4* cfp = od.tcf + (4 * ch) * ns + slot;
          double4 cf[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) cf[u] = cfp[u * ns];
          const int nrs[4] = {nr4.x, nr4.y, nr4.z, nr4.w};
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int ro = nrs[u] & 0xff;
            const cplx s_ = R[ro];
            const cplx g_ = G[ro];
            const double* q = VQ + (nrs[u] >> 8);
            const double csi = cf[u].y * s_.im, csr = cf[u].x * s_.re;
            const double cgi = cf[u].y * g_.im, cgr = cf[u].x * g_.re;
            sl = fma(cf[u].w * q[0], s_.im, fma(cf[u].z * q[1], s_.re, sl));
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const double xr = q[2 + 2 * c], xi = q[3 + 2 * c];
              const double dxr = q[10 + 2 * c], dxi = q[11 + 2 * c];
              Ia[c] = fma(xr, csi, fma(xi, csr, Ia[c]));
              dIa[c] = fma(dxr, csi, fma(dxi, csr, dIa[c]));
              dIa[c] = fma(xr, cgi, fma(xi, cgr, dIa[c]));
            }
          }
          nr4 = nr4n;
        }
        // the 1 << lg pieces of a list sit on aligned adjacent lanes (the partner at distance d
        // is idx ^ d): their partial sums are added with lg DPP quad swaps (lanes i ^ 1, i ^ 2)
        {
          double o;
#define RRQ_ADD_PIECES(v)                    \
  o = dpp_f64<0xB1>(v);                      \
  if (lg == 1 || lg == 2) v += o;            \
  o = dpp_f64<0x4E>(v);                      \
  if (lg == 2) v += o;
          for (int c = 0; c < 4; ++c) {
            RRQ_ADD_PIECES(Ia[c]) RRQ_ADD_PIECES(dIa[c])
          }
          RRQ_ADD_PIECES(sl)
#undef RRQ_ADD_PIECES
        }
        if (!act || piece != 0) continue;
        const double* nu = snu + t * 3;
        // gradient of S^{lm} and its normal derivative: nu'.grad (d_a S^{lm}) is the same
        // ladder combination applied to the table nu'.grad S^{ab}
        cplx g[3], hn[3];
        for (int a = 0; a < 3; ++a) {
          g[a] = dS(R, l, m, a);
          hn[a] = dS(G, l, m, a);
        }
        const double o0 = -som[t * 4], o1 = som[t * 4 + 1], o2 = som[t * 4 + 2], o3 = som[t * 4 + 3];
        const double p0 = -sdom[t * 4], p1 = sdom[t * 4 + 1], p2 = sdom[t * 4 + 2], p3 = sdom[t * 4 + 3];
        cplx Ig[4], dIg[4];
        Ig[0] = mk(0, 0) - (o1 * g[0] + o2 * g[1] + o3 * g[2]);
        Ig[1] = o0 * g[0] + (o2 * g[2] - o3 * g[1]);
        Ig[2] = o0 * g[1] + (o3 * g[0] - o1 * g[2]);
        Ig[3] = o0 * g[2] + (o1 * g[1] - o2 * g[0]);
        dIg[0] = mk(0, 0) - (p1 * g[0] + p2 * g[1] + p3 * g[2]) - (o1 * hn[0] + o2 * hn[1] + o3 * hn[2]);
        dIg[1] = p0 * g[0] + (p2 * g[2] - p3 * g[1]) + o0 * hn[0] + (o2 * hn[2] - o3 * hn[1]);
        dIg[2] = p0 * g[1] + (p3 * g[0] - p1 * g[2]) + o0 * hn[1] + (o3 * hn[0] - o1 * hn[2]);
        dIg[3] = p0 * g[2] + (p1 * g[1] - p2 * g[0]) + o0 * hn[2] + (o1 * hn[1] - o2 * hn[0]);
        double Dq[4], dDq[4];
        for (int c = 0; c < 4; ++c) {
          Dq[c] = -kSqrt2 * kInv4Pi * (Ia[c] + Ig[c].im);
          dDq[c] = -kSqrt2 * kInv4Pi * (dIa[c] + dIg[c].im);
        }
        const double Psi = kSqrt2 * kInv4Pi * (sl - R[tri(l, m)].im * som[t * 4]);
        const double n0_ = nu[0], n1_ = nu[1], n2_ = nu[2];
        double Eq[4];
        Eq[0] = -(n0_ * Dq[1] + n1_ * Dq[2] + n2_ * Dq[3]);
        Eq[1] = Dq[0] * n0_ + (n1_ * Dq[3] - n2_ * Dq[2]);
        Eq[2] = Dq[0] * n1_ + (n2_ * Dq[1] - n0_ * Dq[3]);
        Eq[3] = Dq[0] * n2_ + (n0_ * Dq[2] - n1_ * Dq[1]);
        double* rD = rows + t * L::R4;
        double* rSp = rows + T * L::R4 + t * L::R4;
        double* rS = rows + 2 * T * L::R4 + t * L::R5;
        double* rDp = rows + 2 * T * L::R4 + T * L::R5 + t * L::R4;
        const double sgn[4] = {1.0, -1.0, -1.0, -1.0};
        for (int c = 0; c < 4; ++c) {
          rD[c * NP + lm] = sgn[c] * Dq[c];
          rSp[c * NP + lm] = sgn[c] * Eq[c];
          rDp[c * NP + lm] = sgn[c] * dDq[c];
          rS[(c + 1) * NP + lm] = sgn[c] * Dq[c];
        }
        rS[lm] = Psi;
        if (sself[t] >= 0 && (out.flags & RRQ_F_ONSURF_PV)) {
          const double gh0 = kSqrt2 * g[0].im, gh1 = kSqrt2 * g[1].im, gh2 = kSqrt2 * g[2].im;
          rD[1 * NP + lm] += 0.5 * gh0;
          rD[2 * NP + lm] += 0.5 * gh1;
          rD[3 * NP + lm] += 0.5 * gh2;
          rSp[0 * NP + lm] += 0.5 * (n0_ * gh0 + n1_ * gh1 + n2_ * gh2);
          rSp[1 * NP + lm] += 0.5 * (n1_ * gh2 - n2_ * gh1);
          rSp[2 * NP + lm] += 0.5 * (n2_ * gh0 - n0_ * gh2);
          rSp[3 * NP + lm] += 0.5 * (n0_ * gh1 - n1_ * gh0);
        }
      }
      __syncthreads();
      RRQ_PHASE(4)
      // ---- Step 8 with the density (potentials mode): pair potentials rows . c_K with the
      // patch coefficients c_K = M_K sigma_P, minus the smooth rule over the patch nodes
      if constexpr (POT) {
        // one wave per target: lanes stride over the row entries and the patch nodes, then
        // one wave sum per kernel
        const double* cP = out.pcoef + (int64_t)P * kCoefStride;
        const bool corr = (out.flags & RRQ_F_CORRECTION) != 0;
        const double sc = fr[12];
        for (int t = wv; t < nt; t += BNT / 64) {
          const int64_t k = sids[t * 3];
          const double* xt = sxg + t * 6;
          const double* rD = rows + t * L::R4;
          const double* rSp = rows + T * L::R4 + t * L::R4;
          const double* rS = rows + 2 * T * L::R4 + t * L::R5;
          const double* rDp = rows + 2 * T * L::R4 + T * L::R5 + t * L::R4;
          double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
          for (int i = lane; i < 5 * NP; i += 64) a0 += rS[i] * cP[8 * NP + i];
          for (int i = lane; i < 4 * NP; i += 64) {
            const double cD = cP[i];
            a1 += rD[i] * cD;
            a2 += rSp[i] * cP[4 * NP + i];
            a3 += rDp[i] * cD;
          }
          a0 *= sc;
          a3 /= sc;
          if (corr) {
            const double x0 = xt[0], x1 = xt[1], x2 = xt[2];
            const double nt0 = xt[3], nt1 = xt[4], nt2 = xt[5];
            for (int j = lane; j < Q2; j += 64) {
              if (j == sself[t]) continue;
              const int64_t nj = fresh(n0) + j;
              const double d0 = x0 - pd.node_xyz[nj];
              const double d1 = x1 - pd.node_xyz[pd.N + nj];
              const double d2 = x2 - pd.node_xyz[2 * pd.N + nj];
              const double v0 = pd.node_nrm[nj], v1 = pd.node_nrm[pd.N + nj], v2 = pd.node_nrm[2 * pd.N + nj];
              const double R2 = d0 * d0 + d1 * d1 + d2 * d2;
              const double ri = 1.0 / sqrt(R2), ri2 = ri * ri, ri3 = ri2 * ri;
              const double dn = d0 * v0 + d1 * v1 + d2 * v2;
              const double dnt = d0 * nt0 + d1 * nt1 + d2 * nt2;
              const double f = pd.node_wt[nj] * kInv4Pi * out.dens[nj];
              a0 -= f * ri;
              a1 -= f * (dn * ri3);
              a2 -= f * (-dnt * ri3);
              a3 -= f * (((v0 * nt0 + v1 * nt1 + v2 * nt2) - 3.0 * dn * dnt * ri2) * ri3);
            }
          }
          a0 = wave_sum(a0);
          a1 = wave_sum(a1);
          a2 = wave_sum(a2);
          a3 = wave_sum(a3);
          if (lane < 4 && (out.kmask & (1u << lane))) {
            const double v = lane == 0 ? a0 : (lane == 1 ? a1 : (lane == 2 ? a2 : a3));
            if (!isfinite(v)) {
              atomicAdd(&out.counters[kCNonfinite], 1ull);
              flag_pair(out.pflags, out.counters, k, kFlagNonfinite);
            }
            out.pairpot[k * 4 + lane] = v;
          }
        }
      } else {
        // ---- Step 8 (matrix rows): weights = rows x maps on the four-block 4x4x4 FP64 MFMA.
        // Jobs (group, 16-column tile): group 0 = rD and rDp x M_D (two accumulators sharing
        // the map operand), 1 = rSp x M_Sp, 2 = rS x M_S.  Operand layout: block b = (l % 16)
        // / 4 of lane l takes columns 4b..4b+3 of the tile; lane l supplies A[m = l % 4][k =
        // l / 16] (a target row) and B[k = l / 16][n = l % 4] (a map entry) and receives
        // D[m = l / 16][n = l % 4]: the weight of target l / 16 (of a quad of targets) at
        // column l % 16 of the tile.
        {
          constexpr int NCT = (Q2 + 15) / 16;
          constexpr int TQ = T / 4;
          const double* maps = pd.maps + pd.map_off[P];
          const double sc = fr[12];
          const int am = lane & 3, kr = lane >> 4;
          for (int job = wv; job < 3 * NCT; job += BNT / 64) {
            const int grp = job / NCT, ct = job % NCT;
            const double* M = grp == 0 ? maps : (grp == 1 ? maps + 4 * NP * Q2 : maps + 8 * NP * Q2);
            const int KR = grp == 2 ? 5 * NP : 4 * NP;
            const int NA = grp == 0 ? 2 * TQ : TQ;          // accumulators: (kind, target quad)
            const int bcol = ct * 16 + (lane & 15);
            const bool bval = bcol < Q2;
            double acc[2 * TQ], acc2[2 * TQ];
#pragma unroll
            for (int a = 0; a < 2 * TQ; ++a) acc[a] = acc2[a] = 0.0;
            // 8 k-steps per batch: the map operands of the next batch are loaded before this
            // batch's row operands and MFMAs (8 loads in flight behind the products), and the
            // MFMAs alternate between two partial sums so that consecutive ones do not wait
            // on each other.  Loads are unconditional, at clamped indices: the map operand is
            // zeroed past row KR (so the clamped row entries there add exact zeros), and rows
            // of targets past nt read target 0's row (row m of the product depends on row m
            // of A only, and those rows are not stored).
            const int bc = min(bcol, Q2 - 1);
            double bn[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) bn[u] = M[min(4 * u + kr, KR - 1) * Q2 + bc];
            for (int kb = 0; kb < KR; kb += 32) {
              double bv[8];
#pragma unroll
              for (int u = 0; u < 8; ++u) {
                const int k = kb + 4 * u + kr;
                bv[u] = (bval && k < KR) ? bn[u] : 0.0;
                bn[u] = M[min(k + 32, KR - 1) * Q2 + bc];
              }
#pragma unroll
              for (int a = 0; a < 2 * TQ; ++a) {
                if (a >= NA) break;
                int t = (a % TQ) * 4 + am;
                if (t >= nt) t = 0;
                const double* rowp;
                if (grp == 0)
                  rowp = a < TQ ? rows + t * L::R4 : rows + 2 * T * L::R4 + T * L::R5 + t * L::R4;
                else if (grp == 1) rowp = rows + T * L::R4 + t * L::R4;
                else rowp = rows + 2 * T * L::R4 + t * L::R5;
                double av[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) av[u] = rowp[min(kb + 4 * u + kr, KR - 1)];
#pragma unroll
                for (int u = 0; u < 8; u += 2) {
                  acc[a] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[u], bv[u], acc[a], 0, 0, 0);
                  acc2[a] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[u + 1], bv[u + 1], acc2[a], 0, 0, 0);
                }
              }
            }
#pragma unroll
            for (int a = 0; a < 2 * TQ; ++a) acc[a] += acc2[a];
            if (!bval) continue;
            const int j = bcol;
            const int64_t nj = fresh(n0) + j;
            const double rx = pd.node_xyz[nj], ry = pd.node_xyz[pd.N + nj], rz = pd.node_xyz[2 * pd.N + nj];
            const double v0 = pd.node_nrm[nj], v1 = pd.node_nrm[pd.N + nj], v2 = pd.node_nrm[2 * pd.N + nj];
            const double wj = pd.node_wt[nj] * kInv4Pi;
#pragma unroll
            for (int a = 0; a < 2 * TQ; ++a) {
              if (a >= NA) break;
              const int t = (a % TQ) * 4 + kr;
              const int K = grp == 0 ? (a < TQ ? 1 : 3) : (grp == 1 ? 2 : 0);
              if (t >= nt || !(out.kmask & (1u << K)) || out.w[K] == nullptr) continue;
              const double* xt = sxg + t * 6;
              double val = acc[a];
              if (K == 0) val *= sc;
              else if (K == 3) val /= sc;
              if ((out.flags & RRQ_F_CORRECTION) && j != sself[t]) {
                // smooth-rule kernels from one reciprocal square root: 1/R, then powers
                const double d0 = xt[0] - rx, d1 = xt[1] - ry, d2 = xt[2] - rz;
                const double R2 = d0 * d0 + d1 * d1 + d2 * d2;
                const double ri = 1.0 / sqrt(R2), ri2 = ri * ri, ri3 = ri2 * ri;
                double kv;
                if (K == 0) {
                  kv = ri;
                } else if (K == 1) {
                  kv = (d0 * v0 + d1 * v1 + d2 * v2) * ri3;
                } else {
                  const double nt0 = xt[3], nt1 = xt[4], nt2 = xt[5];
                  const double dnt = d0 * nt0 + d1 * nt1 + d2 * nt2;
                  if (K == 2) {
                    kv = -dnt * ri3;
                  } else {
                    const double dn = d0 * v0 + d1 * v1 + d2 * v2;
                    kv = ((v0 * nt0 + v1 * nt1 + v2 * nt2) - 3.0 * dn * dnt * ri2) * ri3;
                  }
                }
                val -= kv * wj;
              }
              if (!isfinite(val)) {
                atomicAdd(&out.counters[kCNonfinite], 1ull);
                flag_pair(out.pflags, out.counters, sids[t * 3], kFlagNonfinite);
              }
              out.w[K][sids[t * 3 + 2] + j] = val;
            }
          }
        }
      }
    }
  }
  RRQ_PHASE(5)
  RRQ_PHASE_FLUSH
}

#define RRQ_TILE_CASES(X) X(4, 4) X(4, 8) X(5, 4) X(5, 8) X(6, 4) X(6, 8) X(8, 4) X(8, 8) X(10, 4)

size_t tile_lds_bytes(int q, int T) {
  switch (q * 100 + T) {
#define X(Q, T) case Q * 100 + T: return TileLds<Q, T>::bytes;
    RRQ_TILE_CASES(X)
#undef X
  }
  return 0;
}

int tile_supported(int q, int T) { return tile_lds_bytes(q, T) > 0 && tile_lds_bytes(q, T) <= 160 * 1024; }

template <int Q, int TT, bool POT>
static hipError_t launch_tile_case(int grid, const PlanDev& pd, const OrderDev& od,
                                   const TargetsDev& tg, const AssembleOut& out,
                                   const SolveOpts& so, const int4* tiles, const int64_t* qtile,
                                   unsigned long long* qctr, const int64_t* sorted,
                                   hipStream_t st) {
  const size_t lds = TileLds<Q, TT>::bytes;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_pair_tile<Q, TT, POT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL((k_pair_tile<Q, TT, POT>), dim3(grid), dim3(BNT), lds, st, pd, od, tg, out,
                     so, tiles, qtile, qctr, sorted);
  return hipGetLastError();
}

hipError_t launch_pair_tile(int q, int T, bool pot, int grid, const PlanDev& pd,
                            const OrderDev& od, const TargetsDev& tg, const AssembleOut& out,
                            const SolveOpts& so, const int4* tiles, const int64_t* qtile,
                            unsigned long long* qctr, const int64_t* sorted, hipStream_t st) {
  if (tg.nnz <= 0) return hipSuccess;
  switch (q * 100 + T) {
#define X(Q, TT)                                                                              \
  case Q * 100 + TT:                                                                         \
    return pot ? launch_tile_case<Q, TT, true>(grid, pd, od, tg, out, so, tiles, qtile, qctr, \
                                               sorted, st)                                    \
               : launch_tile_case<Q, TT, false>(grid, pd, od, tg, out, so, tiles, qtile,      \
                                                qctr, sorted, st);
    RRQ_TILE_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------------------
// potentials mode: patch coefficients c = maps . sigma_P, per-target sums of the pair
// potentials, and the direct smooth-rule sum over all nodes (small meshes)
// ---------------------------------------------------------------------------------------
__global__ void k_patch_coef(PlanDev pd, const double* dens, double* pcoef) {
  for (int P = blockIdx.x; P < pd.npatch; P += gridDim.x) {
    const int q = pd.order[P], q2 = q * q, nr = 13 * np_of(q);
    const double* M = pd.maps + pd.map_off[P];
    const double* s = dens + pd.node_off[P];
    for (int r = threadIdx.x; r < nr; r += blockDim.x) {
      double acc = 0.0;
      for (int j = 0; j < q2; ++j) acc += M[(int64_t)r * q2 + j] * s[j];
      pcoef[(int64_t)P * kCoefStride + r] = acc;
    }
  }
}

__global__ void k_pot_reduce(TargetsDev tg, uint32_t kmask, const double* pairpot, double* p0,
                             double* p1, double* p2, double* p3) {
  if (input_bad(tg)) return;
  double* Pp[4] = {p0, p1, p2, p3};
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tg.T;
       t += (int64_t)gridDim.x * blockDim.x)
    for (int K = 0; K < 4; ++K) {
      if (!(kmask & (1u << K))) continue;
      double acc = 0.0;
      for (int64_t k = tg.near_ptr[t]; k < tg.near_ptr[t + 1]; ++k) acc += pairpot[k * 4 + K];
      Pp[K][t] = acc;
    }
}

__global__ void k_smooth_direct(PlanDev pd, TargetsDev tg, uint32_t kmask, const double* dens,
                                double* p0, double* p1, double* p2, double* p3) {
  __shared__ double red[4][BNT / 64];
  double* Pp[4] = {p0, p1, p2, p3};
  for (int64_t t = blockIdx.x; t < tg.T; t += gridDim.x) {
    const double x0 = tg.xyz[t], x1 = tg.xyz[tg.T + t], x2 = tg.xyz[2 * tg.T + t];
    const double nt0 = tg.nrm[t], nt1 = tg.nrm[tg.T + t], nt2 = tg.nrm[2 * tg.T + t];
    // the self node is skipped only for an in-range index (this call has no validation word)
    const int sp = tg.self_patch[t];
    const int64_t self = (sp >= 0 && sp < pd.npatch) ? pd.node_off[sp] + tg.self_node[t] : -1;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t j = threadIdx.x; j < pd.N; j += blockDim.x) {
      if (j == self) continue;
      const double d0 = x0 - pd.node_xyz[j], d1 = x1 - pd.node_xyz[pd.N + j],
                   d2 = x2 - pd.node_xyz[2 * pd.N + j];
      const double v0 = pd.node_nrm[j], v1 = pd.node_nrm[pd.N + j], v2 = pd.node_nrm[2 * pd.N + j];
      const double R2 = d0 * d0 + d1 * d1 + d2 * d2;
      const double ri = 1.0 / sqrt(R2), ri2 = ri * ri, ri3 = ri2 * ri;
      const double dn = d0 * v0 + d1 * v1 + d2 * v2;
      const double dnt = d0 * nt0 + d1 * nt1 + d2 * nt2;
      const double f = pd.node_wt[j] * kInv4Pi * dens[j];
      acc[0] += f * ri;
      acc[1] += f * (dn * ri3);
      acc[2] += f * (-dnt * ri3);
      acc[3] += f * (((v0 * nt0 + v1 * nt1 + v2 * nt2) - 3.0 * dn * dnt * ri2) * ri3);
    }
    for (int K = 0; K < 4; ++K) {
      const double v = wave_sum(acc[K]);
      if ((threadIdx.x & 63) == 0) red[K][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4 && (kmask & (1u << threadIdx.x))) {
      double s = 0.0;
      for (int w = 0; w < BNT / 64; ++w) s += red[threadIdx.x][w];
      Pp[threadIdx.x][t] = s;
    }
    __syncthreads();
  }
}

hipError_t launch_patch_coef(const PlanDev& pd, const double* dens, double* pcoef, hipStream_t st) {
  const int g = pd.npatch < 4096 ? pd.npatch : 4096;
  hipLaunchKernelGGL(k_patch_coef, dim3(g > 0 ? g : 1), dim3(256), 0, st, pd, dens, pcoef);
  return hipGetLastError();
}

hipError_t launch_pot_reduce(const TargetsDev& tg, uint32_t kmask, const double* pairpot,
                             double* const* pot, hipStream_t st) {
  if (tg.T <= 0) return hipSuccess;
  int64_t g = (tg.T + 255) / 256;
  hipLaunchKernelGGL(k_pot_reduce, dim3((unsigned)(g < 65535 ? g : 65535)), dim3(256), 0, st, tg,
                     kmask, pairpot, pot[0], pot[1], pot[2], pot[3]);
  return hipGetLastError();
}

hipError_t launch_smooth_direct(const PlanDev& pd, const TargetsDev& tg, uint32_t kmask,
                                const double* dens, double* const* pot, hipStream_t st) {
  if (tg.T <= 0) return hipSuccess;
  const int64_t g = tg.T < 65535 ? tg.T : 65535;
  hipLaunchKernelGGL(k_smooth_direct, dim3((unsigned)g), dim3(BNT), 0, st, pd, tg, kmask, dens,
                     pot[0], pot[1], pot[2], pot[3]);
  return hipGetLastError();
}

}  // namespace rrq

#ifdef RRQ_PHASE_TIMERS
// profiling build only: the per-phase sums of the tile kernel's timers (8 values), and their
// reset; both synchronise with the device
extern "C" int rrq_phase_read(unsigned long long* host8) {
  return (int)hipMemcpyFromSymbol(host8, HIP_SYMBOL(rrq::g_tile_phase), 8 * sizeof(unsigned long long));
}
extern "C" int rrq_phase_reset() {
  const unsigned long long z[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  return (int)hipMemcpyToSymbol(HIP_SYMBOL(rrq::g_tile_phase), z, sizeof(z));
}
#endif
