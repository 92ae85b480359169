// Host runtime behind the C ABI of include/rrq.h: plan memory, constant tables, argument
// validation and kernel launches.
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "rrq_internal.h"

using namespace rrq;

namespace {

bool supported_order(int q) {
  for (int i = 0; i < kNumOrders; ++i)
    if (kOrders[i] == q) return true;
  return false;
}

template <typename T>
hipError_t dalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  return hipMalloc((void**)p, n * sizeof(T));
}

}  // namespace

struct rrq_plan {
  int32_t P = 0;
  int64_t N = 0, E = 0;
  std::vector<int32_t> order_h;
  std::vector<int64_t> node_off_h, edge_off_h;
  rrq_options opt{};
  // device copies / products
  int32_t* order_d = nullptr;
  int64_t* node_off_d = nullptr;
  int64_t* edge_off_d = nullptr;
  double* node_xyz_d = nullptr;   // [3][N]
  double* node_nrm_d = nullptr;
  double* node_wt_d = nullptr;
  double* frame_d = nullptr;
  double* node_loc_d = nullptr;
  double* edge_loc_d = nullptr;
  double* edge_tan_d = nullptr;
  double* edge_coef_d = nullptr;
  double* edge_chord_d = nullptr;  // [P][4][6]
  double* maps_d = nullptr;
  int64_t* map_off_d = nullptr;
  double* tabs_d = nullptr;
  int64_t* tab_off_d = nullptr;
  double* fit_ws_d = nullptr;
  double* fitcond_d = nullptr;    // [P][2]
  int64_t fit_ws_per_block = 0;
  int fit_blocks = 0;
  // per order
  std::vector<int32_t> patches_h[kMaxQ + 1];
  int32_t* patches_d[kMaxQ + 1] = {};
  int32_t* perm_d = nullptr;    // patches grouped by order (kOrders order)
  float* mlp_d = nullptr;       // learned-guess network (ABI parameter layout)
  bool has_mlp = false;
  BinOrders bin_orders{};
  OrderDev od[kMaxQ + 1] = {};
  std::vector<void*> const_bufs;
  double rho_far[kMaxQ + 1] = {};
  int tile[kMaxQ + 1] = {};     // targets per tile of the batched form, per order
  int grid[kMaxQ + 1] = {};     // workgroups of the batched kernel, per order

  PlanDev dev() const {
    PlanDev d;
    d.npatch = P;
    d.N = N;
    d.E = E;
    d.order = order_d;
    d.node_off = node_off_d;
    d.edge_off = edge_off_d;
    d.node_xyz = node_xyz_d;
    d.node_nrm = node_nrm_d;
    d.node_wt = node_wt_d;
    d.frame = frame_d;
    d.node_loc = node_loc_d;
    d.edge_loc = edge_loc_d;
    d.edge_tan = edge_tan_d;
    d.edge_coef = edge_coef_d;
    d.edge_chord = edge_chord_d;
    d.maps = maps_d;
    d.map_off = map_off_d;
    d.tabs = tabs_d;
    d.tab_off = tab_off_d;
    d.mlp = has_mlp ? mlp_d : nullptr;
    d.fitcond = fitcond_d;
    return d;
  }
};

static void plan_free(rrq_plan* p) {
  if (!p) return;
  void* ptrs[] = {p->order_d, p->node_off_d, p->edge_off_d, p->node_xyz_d, p->node_nrm_d,
                  p->node_wt_d, p->frame_d, p->node_loc_d, p->edge_loc_d, p->edge_tan_d,
                  p->edge_coef_d, p->maps_d, p->map_off_d, p->tabs_d, p->tab_off_d,
                  p->fit_ws_d, p->perm_d, p->mlp_d, p->fitcond_d, p->edge_chord_d};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  for (int q = 0; q <= kMaxQ; ++q)
    if (p->patches_d[q]) (void)hipFree(p->patches_d[q]);
  for (void* b : p->const_bufs) (void)hipFree(b);
  delete p;
}

static rrq_status upload_consts(rrq_plan* p, int q) {
  OrderTables T = build_order_tables(q, 2 * q);
  auto up = [&](const void* src, size_t bytes, void** dst) -> bool {
    if (hipMalloc(dst, bytes ? bytes : 8) != hipSuccess) return false;
    p->const_bufs.push_back(*dst);
    return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
  };
  OrderDev& o = p->od[q];
  o.q = q;
  o.pt = T.pt;
  o.np = T.np;
  o.njk = T.njk;
  void* b;
  if (!up(T.gl_t.data(), T.gl_t.size() * 8, &b)) return RRQ_ERR_OOM;
  o.gl_t = (const double*)b;
  if (!up(T.gl_w.data(), T.gl_w.size() * 8, &b)) return RRQ_ERR_OOM;
  o.gl_w = (const double*)b;
  // least-squares row weights: the q-point GL weights, or ones for the unweighted fit
  if (p->opt.ls_unweighted) std::fill(T.glq_w.begin(), T.glq_w.end(), 1.0);
  if (!up(T.glq_w.data(), T.glq_w.size() * 8, &b)) return RRQ_ERR_OOM;
  o.glq_w = (const double*)b;
  if (!up(T.LT.data(), T.LT.size() * 8, &b)) return RRQ_ERR_OOM;
  o.LT = (const double*)b;
  if (!up(T.DP.data(), T.DP.size() * 8, &b)) return RRQ_ERR_OOM;
  o.DP = (const double*)b;
  if (!up(T.lag_m1.data(), T.lag_m1.size() * 8, &b)) return RRQ_ERR_OOM;
  o.lag_m1 = (const double*)b;
  if (!up(T.bary.data(), T.bary.size() * 8, &b)) return RRQ_ERR_OOM;
  o.bary = (const double*)b;
  if (!up(T.bary1.data(), T.bary1.size() * 8, &b)) return RRQ_ERR_OOM;
  o.bary1 = (const double*)b;
  if (!up(T.dlp_ptr.data(), T.dlp_ptr.size() * 4, &b)) return RRQ_ERR_OOM;
  o.dlp_ptr = (const int32_t*)b;
  if (!up(T.dlp.data(), T.dlp.size() * sizeof(Term), &b)) return RRQ_ERR_OOM;
  o.dlp = (const Term*)b;
  if (!up(T.slp_ptr.data(), T.slp_ptr.size() * 4, &b)) return RRQ_ERR_OOM;
  o.slp_ptr = (const int32_t*)b;
  if (!up(T.slp.data(), T.slp.size() * sizeof(Term), &b)) return RRQ_ERR_OOM;
  o.slp = (const Term*)b;
  for (int32_t v : T.mrg_ptr)
    if (v < 0) return RRQ_ERR_DEVICE;   // term tables inconsistent (cannot happen)
  if (!up(T.mrg_ptr.data(), T.mrg_ptr.size() * 4, &b)) return RRQ_ERR_OOM;
  o.mrg_ptr = (const int32_t*)b;
  if (!up(T.mrg.data(), T.mrg.size() * sizeof(Term2), &b)) return RRQ_ERR_OOM;
  o.mrg = (const Term2*)b;
  if (!up(T.tslot.data(), T.tslot.size() * 4, &b)) return RRQ_ERR_OOM;
  o.tslot = (const int32_t*)b;
  o.nslot = (int)T.tslot.size();
  if (!up(T.tlen.data(), T.tlen.size() * 4, &b)) return RRQ_ERR_OOM;
  o.tlen = (const int32_t*)b;
  if (!up(T.tnr.data(), T.tnr.size() * 4, &b)) return RRQ_ERR_OOM;
  o.tnr = (const int4*)b;
  if (!up(T.tcf.data(), T.tcf.size() * 8, &b)) return RRQ_ERR_OOM;
  o.tcf = (const double4*)b;
  return RRQ_OK;
}

static rrq_status check_surface(const rrq_surface* s) {
  if (!s || s->npatch <= 0 || !s->order_host || !s->order || !s->node_off || !s->node_xyz ||
      !s->node_nrm || !s->node_wt || !s->edge_off || !s->edge_xyz || s->nnode <= 0 ||
      s->nedge <= 0)
    return RRQ_ERR_ARG;
  int64_t N = 0, E = 0;
  for (int P = 0; P < s->npatch; ++P) {
    const int q = s->order_host[P];
    if (!supported_order(q)) return RRQ_ERR_UNSUPPORTED;
    N += (int64_t)q * q;
    E += 8LL * q;
  }
  if (N != s->nnode || E != s->nedge) return RRQ_ERR_ARG;
  return RRQ_OK;
}

__global__ void k_copy3(const double* a, const double* b, const double* c, double* A, double* B,
                        double* C, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * n;
       i += (int64_t)gridDim.x * blockDim.x) {
    A[i] = a[i];
    B[i] = b[i];
    if (i < n) C[i] = c[i];
  }
}

// Source-only data in two parts: the geometry (frames, local nodes, edge interpolants), which
// the root and near-edge pre-passes need, and the maps and edge tables, which only the tile
// kernels need (a captured step runs the fits beside the edge tables and the pre-passes).
static rrq_status run_geometry(rrq_plan* p, const rrq_surface* s, hipStream_t st) {
  // plan copies of the smooth-rule data used by the correction (a kernel, not a memcpy, so
  // that the step can be captured into a graph)
  {
    int64_t g = (3 * p->N + 255) / 256;
    hipLaunchKernelGGL(k_copy3, dim3((unsigned)(g < 65535 ? g : 65535)), dim3(256), 0, st,
                       s->node_xyz, s->node_nrm, s->node_wt, p->node_xyz_d, p->node_nrm_d,
                       p->node_wt_d, p->N);
    if (hipGetLastError() != hipSuccess) return RRQ_ERR_DEVICE;
  }
  PlanDev pd = p->dev();
  rrq_surface sd = *s;
  sd.node_off = p->node_off_d;
  sd.edge_off = p->edge_off_d;
  for (int qi = 0; qi < kNumOrders; ++qi) {
    const int q = kOrders[qi];
    const int cnt = (int)p->patches_h[q].size();
    if (!cnt) continue;
    if (launch_geometry(pd, sd, p->od[q], p->patches_d[q], cnt, st) != hipSuccess)
      return RRQ_ERR_DEVICE;
  }
  return RRQ_OK;
}

static rrq_status run_edge_tables(rrq_plan* p, hipStream_t st) {
  PlanDev pd = p->dev();
  for (int qi = 0; qi < kNumOrders; ++qi) {
    const int q = kOrders[qi];
    const int cnt = (int)p->patches_h[q].size();
    if (cnt && launch_edge_tables(pd, p->od[q], p->patches_d[q], cnt, st) != hipSuccess)
      return RRQ_ERR_DEVICE;
  }
  return RRQ_OK;
}

static rrq_status run_fits(rrq_plan* p, hipStream_t st) {
  PlanDev pd = p->dev();
  for (int qi = 0; qi < kNumOrders; ++qi) {
    const int q = kOrders[qi];
    const int cnt = (int)p->patches_h[q].size();
    if (cnt && launch_fit(pd, p->od[q], p->patches_d[q], cnt, p->fit_ws_d, p->fit_ws_per_block,
                          p->fit_blocks, st) != hipSuccess)
      return RRQ_ERR_DEVICE;
  }
  return RRQ_OK;
}

static rrq_status run_maps(rrq_plan* p, hipStream_t st) {
  const rrq_status r = run_edge_tables(p, st);
  return r == RRQ_OK ? run_fits(p, st) : r;
}

static rrq_status run_fit(rrq_plan* p, const rrq_surface* s, hipStream_t st) {
  rrq_status r = run_geometry(p, s, st);
  return r == RRQ_OK ? run_maps(p, st) : r;
}

extern "C" {

const char* rrq_status_string(rrq_status s) {
  switch (s) {
    case RRQ_OK: return "ok";
    case RRQ_ERR_ARG: return "invalid argument";
    case RRQ_ERR_DEVICE: return "device error";
    case RRQ_ERR_OOM: return "out of device memory";
    case RRQ_ERR_ILLCONDITIONED: return "ill-conditioned or non-finite patch fit";
    case RRQ_ERR_UNSUPPORTED: return "unsupported order, size or option";
    case RRQ_ERR_BUFFER: return "buffer too small";
    case RRQ_ERR_NONFINITE: return "non-finite outputs";
  }
  return "unknown status";
}

rrq_status rrq_plan_create(const rrq_surface* s, const rrq_options* opts, void* stream,
                           rrq_plan** out) {
  if (!out) return RRQ_ERR_ARG;
  *out = nullptr;
  rrq_status cs = check_surface(s);
  if (cs != RRQ_OK) return cs;
  rrq_plan* p = new (std::nothrow) rrq_plan();
  if (!p) return RRQ_ERR_OOM;
  if (opts) p->opt = *opts;
  if (p->opt.newton_tol <= 0) p->opt.newton_tol = 1e-14;
  if (p->opt.newton_maxit <= 0) p->opt.newton_maxit = 60;
  if (p->opt.ls_unweighted != 0 && p->opt.ls_unweighted != 1) {
    delete p;
    return RRQ_ERR_ARG;
  }
  if ((p->opt.ptilde_factor != 0 && p->opt.ptilde_factor != 2) || p->opt.u_rule != 0) {
    delete p;
    return RRQ_ERR_UNSUPPORTED;
  }
  // the near-edge kernels' panel capacity is sized for the default rho_far of each order
  if (p->opt.rho_far > 0)
    for (int P = 0; P < s->npatch; ++P)
      if (p->opt.rho_far > pow(10.0, 8.0 / (2 * s->order_host[P]))) {
        delete p;
        return RRQ_ERR_UNSUPPORTED;
      }
  if (p->opt.tile_targets != 0 && p->opt.tile_targets != 4 && p->opt.tile_targets != 8) {
    delete p;
    return RRQ_ERR_UNSUPPORTED;
  }
  for (int q = 0; q <= kMaxQ; ++q) p->tile[q] = p->opt.tile_targets > 0 ? p->opt.tile_targets : 4;
  if (p->opt.grid < 0 || p->opt.grid > (1 << 20)) {
    delete p;
    return RRQ_ERR_ARG;
  }
  for (int q = 0; q <= kMaxQ; ++q) p->grid[q] = p->opt.grid > 0 ? p->opt.grid : 2048;
  p->P = s->npatch;
  p->N = s->nnode;
  p->E = s->nedge;
  p->order_h.assign(s->order_host, s->order_host + s->npatch);
  p->node_off_h.resize(p->P + 1);
  p->edge_off_h.resize(p->P + 1);
  std::vector<int64_t> map_off(p->P + 1), tab_off(p->P + 1);
  p->node_off_h[0] = p->edge_off_h[0] = map_off[0] = tab_off[0] = 0;
  int64_t maxws = 0;
  for (int P = 0; P < p->P; ++P) {
    const int q = p->order_h[P];
    p->node_off_h[P + 1] = p->node_off_h[P] + (int64_t)q * q;
    p->edge_off_h[P + 1] = p->edge_off_h[P] + 8LL * q;
    map_off[P + 1] = map_off[P] + map_doubles(q);
    tab_off[P + 1] = tab_off[P] + tab_doubles(q);
    p->patches_h[q].push_back(P);
    maxws = std::max(maxws, fit_ws_doubles(q));
  }
  hipStream_t st = (hipStream_t)stream;
  bool ok = true;
  ok &= dalloc(&p->order_d, p->P) == hipSuccess;
  ok &= dalloc(&p->node_off_d, p->P + 1) == hipSuccess;
  ok &= dalloc(&p->edge_off_d, p->P + 1) == hipSuccess;
  ok &= dalloc(&p->node_xyz_d, 3 * p->N) == hipSuccess;
  ok &= dalloc(&p->node_nrm_d, 3 * p->N) == hipSuccess;
  ok &= dalloc(&p->node_wt_d, p->N) == hipSuccess;
  ok &= dalloc(&p->frame_d, (size_t)p->P * kFrame) == hipSuccess;
  ok &= dalloc(&p->node_loc_d, 6 * p->N) == hipSuccess;
  ok &= dalloc(&p->edge_loc_d, 3 * p->E) == hipSuccess;
  ok &= dalloc(&p->edge_tan_d, 3 * p->E) == hipSuccess;
  ok &= dalloc(&p->edge_coef_d, 3 * p->E) == hipSuccess;
  ok &= dalloc(&p->edge_chord_d, 24 * (size_t)p->P) == hipSuccess;
  ok &= dalloc(&p->maps_d, map_off[p->P]) == hipSuccess;
  ok &= dalloc(&p->map_off_d, p->P + 1) == hipSuccess;
  ok &= dalloc(&p->tabs_d, tab_off[p->P]) == hipSuccess;
  ok &= dalloc(&p->tab_off_d, p->P + 1) == hipSuccess;
  {
    std::vector<int32_t> perm;
    for (int qi = 0; qi < kNumOrders; ++qi) {
      p->bin_orders.off[qi] = (int32_t)perm.size();
      perm.insert(perm.end(), p->patches_h[kOrders[qi]].begin(), p->patches_h[kOrders[qi]].end());
    }
    p->bin_orders.off[kNumOrders] = (int32_t)perm.size();
    ok &= dalloc(&p->perm_d, p->P) == hipSuccess;
    if (ok) ok &= hipMemcpy(p->perm_d, perm.data(), perm.size() * 4, hipMemcpyHostToDevice) ==
                  hipSuccess;
  }
  // persistent fit workgroups: fewer than two per CU, so that in a captured step the kernels
  // of the other branch (edge tables, binning, pre-passes) find room beside them
  p->fit_blocks = std::min(p->P, 384);
  p->fit_ws_per_block = maxws;
  ok &= dalloc(&p->fit_ws_d, (size_t)maxws * p->fit_blocks) == hipSuccess;
  ok &= dalloc(&p->fitcond_d, 2 * (size_t)p->P) == hipSuccess;
  for (int q = 0; q <= kMaxQ && ok; ++q)
    if (!p->patches_h[q].empty()) {
      ok &= dalloc(&p->patches_d[q], p->patches_h[q].size()) == hipSuccess;
      ok &= hipMemcpy(p->patches_d[q], p->patches_h[q].data(), p->patches_h[q].size() * 4,
                      hipMemcpyHostToDevice) == hipSuccess;
      if (ok && upload_consts(p, q) != RRQ_OK) ok = false;
      p->rho_far[q] = p->opt.rho_far > 0 ? p->opt.rho_far : pow(10.0, 8.0 / (2 * q));
    }
  if (!ok) {
    plan_free(p);
    return RRQ_ERR_OOM;
  }
  ok &= hipMemcpy(p->order_d, p->order_h.data(), p->P * 4, hipMemcpyHostToDevice) == hipSuccess;
  ok &= hipMemcpy(p->node_off_d, p->node_off_h.data(), (p->P + 1) * 8, hipMemcpyHostToDevice) ==
        hipSuccess;
  ok &= hipMemcpy(p->edge_off_d, p->edge_off_h.data(), (p->P + 1) * 8, hipMemcpyHostToDevice) ==
        hipSuccess;
  ok &= hipMemcpy(p->map_off_d, map_off.data(), (p->P + 1) * 8, hipMemcpyHostToDevice) ==
        hipSuccess;
  ok &= hipMemcpy(p->tab_off_d, tab_off.data(), (p->P + 1) * 8, hipMemcpyHostToDevice) ==
        hipSuccess;
  if (!ok) {
    plan_free(p);
    return RRQ_ERR_DEVICE;
  }
  rrq_status r = run_fit(p, s, st);
  if (r != RRQ_OK) {
    plan_free(p);
    return r;
  }
  *out = p;
  return RRQ_OK;
}

rrq_status rrq_plan_refit(rrq_plan* p, const rrq_surface* s, void* stream) {
  if (!p) return RRQ_ERR_ARG;
  rrq_status cs = check_surface(s);
  if (cs != RRQ_OK) return cs;
  if (s->npatch != p->P || s->nnode != p->N || s->nedge != p->E) return RRQ_ERR_ARG;
  for (int P = 0; P < p->P; ++P)
    if (s->order_host[P] != p->order_h[P]) return RRQ_ERR_ARG;
  return run_fit(p, s, (hipStream_t)stream);
}

rrq_status rrq_plan_destroy(rrq_plan* p) {
  if (!p) return RRQ_ERR_ARG;
  (void)hipDeviceSynchronize();
  plan_free(p);
  return RRQ_OK;
}

static rrq_status check_targets(const rrq_plan* p, const rrq_targets* tg) {
  if (!p || !tg || tg->ntarget < 0 || tg->nnz < 0) return RRQ_ERR_ARG;
  // tile starts are 32-bit pair positions
  if (tg->nnz >= (int64_t(1) << 31)) return RRQ_ERR_UNSUPPORTED;
  if (tg->ntarget > 0 && (!tg->xyz || !tg->nrm || !tg->self_patch || !tg->self_node ||
                          !tg->near_ptr))
    return RRQ_ERR_ARG;
  if (tg->nnz > 0 && !tg->near_patch) return RRQ_ERR_ARG;
  return RRQ_OK;
}

static TargetsDev tdev(const rrq_targets* tg, const unsigned* bad = nullptr) {
  TargetsDev t;
  t.bad = bad;
  t.T = tg->ntarget;
  t.nnz = tg->nnz;
  t.xyz = tg->xyz;
  t.nrm = tg->nrm;
  t.self_patch = tg->self_patch;
  t.self_node = tg->self_node;
  t.near_ptr = tg->near_ptr;
  t.near_patch = tg->near_patch;
  return t;
}

// workspace layout: owner[nnz] i64 | counters[kNumCounters] u64 | bad u32 | pflags[nnz] u32 |
// cnt[P] i32 | fill[P] i32 |
// start[P+1] i64 | tstart[P+1] i64 | ntiles i64 | qtile[orders+1] i64, qctr[orders][xcds] u64 |
// sorted[nnz] i64 | tiles[nnz/4 + P + 1] int4 | scan partials | root[4 nnz] double2 |
// nearf[4 nnz] u8 | pairpot[nnz][4] f64 | plocal[nnz][9] f64 | ptd[nnz][16] f64 |
// pti[nnz][4] i64 | pcoef[P][kCoefStride] f64 |
// nlist[4 nnz] i64 |
// lamg[4 nnz][lam_stride] f64 (near-edge moments; lam_stride = 2 ptilde_max + 1 >= 5; before
// them, the root passes' Newton and retry lists, 4 nnz i64 each)
struct WsLayout {
  size_t owner, counters, bad, pflags, cnt, fill, start, tstart, ntiles, queue, sorted, tiles,
      part, root, nearf, pairpot, plocal, ptd, pti, pcoef, nlist, lamg, total;
};
static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }
static WsLayout ws_layout(int64_t nnz, int P, int lam_stride) {
  const size_t n = (size_t)(nnz > 0 ? nnz : 1);
  WsLayout w;
  size_t o = 0;
  w.owner = o; o = al(o + n * 8);
  w.counters = o; o = al(o + 8 * kNumCounters);
  w.bad = o; o = al(o + 4);
  w.pflags = o; o = al(o + n * 4);
  w.cnt = o; o = al(o + (size_t)P * 4);
  w.fill = o; o = al(o + (size_t)P * 4);
  w.start = o; o = al(o + (size_t)(P + 1) * 8);
  w.tstart = o; o = al(o + (size_t)(P + 1) * 8);
  w.ntiles = o; o = al(o + 8);
  w.queue = o; o = al(o + 8 * (kNumOrders + 1 + kNumOrders * kXcds));
  w.sorted = o; o = al(o + n * 8);
  w.tiles = o; o = al(o + (n / 4 + (size_t)P + 1) * 16);
  w.part = o; o = al(o + (size_t)scan_partials((int64_t)n) * 8);
  w.root = o; o = al(o + 4 * n * 16);
  w.nearf = o; o = al(o + 4 * n);
  w.pairpot = o; o = al(o + 4 * n * 8);
  w.plocal = o; o = al(o + 9 * n * 8);
  w.ptd = o; o = al(o + 16 * n * 8);
  w.pti = o; o = al(o + 4 * n * 8);
  w.pcoef = o; o = al(o + (size_t)P * kCoefStride * 8);
  w.nlist = o; o = al(o + 4 * n * 8);
  w.lamg = o; o = al(o + 4 * n * (size_t)lam_stride * 8);
  w.total = o;
  return w;
}
// doubles per slot of the near-edge moments: lambda^(1), lambda^(3) at the largest order's
// ptilde edge nodes, and the Omega_0 part
static int lam_stride_of(const rrq_plan* p) {
  int qmax = 1;
  for (int q = 0; q <= kMaxQ; ++q)
    if (!p->patches_h[q].empty()) qmax = q;
  return 2 * (2 * qmax) + 1;
}
static WsLayout ws_layout(const rrq_plan* p, int64_t nnz) {
  return ws_layout(nnz, p->P, lam_stride_of(p));
}
static size_t ws_bytes(const rrq_plan* p, int64_t nnz) { return ws_layout(p, nnz).total; }

rrq_status rrq_plan_fit_condition(const rrq_plan* p, double* cond, void* stream) {
  if (!p || !cond) return RRQ_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  if (hipMemcpyAsync(cond, p->fitcond_d, 2 * (size_t)p->P * sizeof(double), hipMemcpyDeviceToHost,
                     st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return RRQ_ERR_DEVICE;
  return RRQ_OK;
}

rrq_status rrq_plan_patch_flags(const rrq_plan* p, double max_cond, int32_t* flags,
                                void* stream) {
  if (!p || !flags) return RRQ_ERR_ARG;
  const double lim = max_cond > 0 ? max_cond : 1e9;
  hipStream_t st = (hipStream_t)stream;
  int32_t* dflags = nullptr;
  if (dalloc(&dflags, p->P) != hipSuccess) return RRQ_ERR_OOM;
  std::vector<double> cond(2 * (size_t)p->P);
  const bool ok = launch_patch_check(p->dev(), dflags, st) == hipSuccess &&
                  hipMemcpyAsync(flags, dflags, (size_t)p->P * 4, hipMemcpyDeviceToHost, st) ==
                      hipSuccess &&
                  hipMemcpyAsync(cond.data(), p->fitcond_d, cond.size() * sizeof(double),
                                 hipMemcpyDeviceToHost, st) == hipSuccess &&
                  hipStreamSynchronize(st) == hipSuccess;
  (void)hipFree(dflags);
  if (!ok) return RRQ_ERR_DEVICE;
  bool any = false;
  for (int P = 0; P < p->P; ++P) {
    int32_t f = flags[P] ? 4 : 0;
    // a NaN estimate is flagged too (!(c <= lim))
    if (!(cond[2 * (size_t)P] <= lim)) f |= 1;
    if (!(cond[2 * (size_t)P + 1] <= lim)) f |= 2;
    flags[P] = f;
    any |= f != 0;
  }
  return any ? RRQ_ERR_ILLCONDITIONED : RRQ_OK;
}

rrq_status rrq_weights_size(const rrq_plan* p, const rrq_targets* tg, int64_t* nweights,
                            void* stream) {
  rrq_status c = check_targets(p, tg);
  if (c != RRQ_OK) return c;
  if (!nweights) return RRQ_ERR_ARG;
  *nweights = 0;
  hipStream_t st = (hipStream_t)stream;
  std::vector<int64_t> ptr((size_t)tg->ntarget + 1);
  std::vector<int32_t> np((size_t)(tg->nnz > 0 ? tg->nnz : 1));
  if (hipMemcpyAsync(ptr.data(), tg->near_ptr, ptr.size() * 8, hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      (tg->nnz > 0 && hipMemcpyAsync(np.data(), tg->near_patch, (size_t)tg->nnz * 4,
                                     hipMemcpyDeviceToHost, st) != hipSuccess) ||
      hipStreamSynchronize(st) != hipSuccess)
    return RRQ_ERR_DEVICE;
  if (ptr[0] != 0 || ptr[(size_t)tg->ntarget] != tg->nnz) return RRQ_ERR_ARG;
  for (int64_t t = 0; t < tg->ntarget; ++t)
    if (ptr[(size_t)t] > ptr[(size_t)t + 1]) return RRQ_ERR_ARG;
  int64_t n = 0;
  for (int64_t k = 0; k < tg->nnz; ++k) {
    const int32_t P = np[(size_t)k];
    if (P < 0 || P >= p->P) return RRQ_ERR_ARG;
    n += (int64_t)p->order_h[P] * p->order_h[P];
  }
  *nweights = n;
  return RRQ_OK;
}

rrq_status rrq_workspace_size(const rrq_plan* p, const rrq_targets* tg, size_t* bytes) {
  if (!bytes) return RRQ_ERR_ARG;
  rrq_status c = check_targets(p, tg);
  if (c != RRQ_OK) return c;
  *bytes = ws_bytes(p, tg->nnz);
  return RRQ_OK;
}

rrq_status rrq_pair_offsets(const rrq_plan* p, const rrq_targets* tg, int64_t* pair_off,
                            void* workspace, size_t workspace_bytes, int64_t* nweights,
                            void* stream) {
  rrq_status c = check_targets(p, tg);
  if (c != RRQ_OK) return c;
  if (!pair_off || !workspace) return RRQ_ERR_ARG;
  if (workspace_bytes < ws_bytes(p, tg->nnz)) return RRQ_ERR_BUFFER;
  hipStream_t st = (hipStream_t)stream;
  const WsLayout wl = ws_layout(p, tg->nnz);
  int64_t* part = (int64_t*)((char*)workspace + wl.part);
  unsigned* bad = (unsigned*)((char*)workspace + wl.bad);
  const TargetsDev td = tdev(tg, bad);
  if (launch_validate(p->dev(), td, nullptr, 0, bad, nullptr, st) != hipSuccess)
    return RRQ_ERR_DEVICE;
  if (nweights) {
    unsigned hbad = 0;
    if (hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return RRQ_ERR_DEVICE;
    if (hbad) return RRQ_ERR_ARG;
  }
  if (launch_pair_offsets(p->dev(), td, pair_off, part, st) != hipSuccess)
    return RRQ_ERR_DEVICE;
  if (nweights) {
    if (hipMemcpyAsync(nweights, pair_off + tg->nnz, 8, hipMemcpyDeviceToHost, st) != hipSuccess)
      return RRQ_ERR_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return RRQ_ERR_DEVICE;
  }
  return RRQ_OK;
}

// Streams and events of the per-order branches of a captured step (owned by the capture).
struct OrderBranches {
  hipStream_t stream[kNumOrders];
  hipEvent_t fork;
  hipEvent_t join[kNumOrders];
  // the root passes on stream[0] beside the binning and the per-pair target data
  hipEvent_t root_fork, root_join;
};

// Timing events around each order's tile kernel (autotuner and statistics).
struct OrderEvents {
  hipEvent_t e[kNumOrders][2] = {};
  hipError_t record(int qi, int which, hipStream_t st) {
    if (!e[qi][which]) {
      const hipError_t c = hipEventCreate(&e[qi][which]);
      if (c != hipSuccess) return c;
    }
    return hipEventRecord(e[qi][which], st);
  }
  float elapsed(int qi) const {
    float ms = 0.f;
    if (e[qi][0] && e[qi][1] && hipEventElapsedTime(&ms, e[qi][0], e[qi][1]) == hipSuccess)
      return ms;
    return 0.f;
  }
  ~OrderEvents() {
    for (auto& p : e)
      for (hipEvent_t x : p)
        if (x) (void)hipEventDestroy(x);
  }
};

// Assembly of the near pairs: weights (outs) or, with a density, the potentials (pots).
static rrq_status run_pairs(const rrq_plan* p, const rrq_targets* tg, uint32_t kmask,
                            uint32_t flags, double* const* outs, int64_t out_len,
                            const int64_t* pair_off, const double* density, double* const* pots,
                            uint32_t* pair_flags, void* workspace, hipStream_t st,
                            rrq_stats* stats, hipEvent_t maps_ready = nullptr,
                            const OrderBranches* branches = nullptr,
                            float* order_ms = nullptr) {
  const bool pot = pots != nullptr;
  float order_ms_local[kNumOrders] = {};
  if (stats && !order_ms && !(flags & RRQ_F_PLAIN)) order_ms = order_ms_local;
  const WsLayout wl = ws_layout(p, tg->nnz);
  char* wb = (char*)workspace;
  int64_t* owner = (int64_t*)(wb + wl.owner);
  unsigned long long* counters = (unsigned long long*)(wb + wl.counters);
  unsigned* bad = (unsigned*)(wb + wl.bad);
  uint32_t* pflags = pair_flags ? pair_flags : (uint32_t*)(wb + wl.pflags);
  TargetsDev td = tdev(tg, bad);
  // device check of the inputs first (it clears the counters); every later kernel returns at
  // once if it failed
  if (launch_validate(p->dev(), td, pot ? nullptr : pair_off, out_len, bad, counters, st) !=
      hipSuccess)
    return RRQ_ERR_DEVICE;
  if (launch_owner(td, owner, pflags, st) != hipSuccess) return RRQ_ERR_DEVICE;
  AssembleOut ao;
  for (int K = 0; K < 4; ++K) ao.w[K] = (!pot && (kmask & (1u << K))) ? outs[K] : nullptr;
  ao.kmask = kmask;
  ao.flags = flags;
  ao.pair_off = pair_off;
  ao.owner = owner;
  ao.counters = counters;
  ao.pflags = pflags;
  ao.root = nullptr;
  ao.nearf = nullptr;
  ao.lamg = nullptr;
  ao.ptd = nullptr;
  ao.pti = nullptr;
  ao.lam_stride = 0;
  ao.dens = density;
  ao.pcoef = pot ? (const double*)(wb + wl.pcoef) : nullptr;
  ao.pairpot = pot ? (double*)(wb + wl.pairpot) : nullptr;
  PlanDev pd = p->dev();
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (stats) {
    if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess)
      return RRQ_ERR_DEVICE;
  }
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int i = 0; i < 2; ++i)
        if (e[i]) (void)hipEventDestroy(e[i]);
    }
  } evg{ev};
  if (flags & RRQ_F_PLAIN) {
    if (maps_ready && hipStreamWaitEvent(st, maps_ready, 0) != hipSuccess) return RRQ_ERR_DEVICE;
    if (stats && hipEventRecord(ev[0], st) != hipSuccess) return RRQ_ERR_DEVICE;
    for (int qi = 0; qi < kNumOrders; ++qi) {
      const int q = kOrders[qi];
      if (p->patches_h[q].empty()) continue;
      SolveOpts so{p->rho_far[q], p->opt.newton_tol, p->opt.newton_maxit};
      if (launch_pair_plain(q, pd, p->od[q], td, ao, so, st) != hipSuccess) return RRQ_ERR_DEVICE;
    }
  } else {
    // targets per tile of each order (the largest supported one not above the plan's choice)
    BinOrders bo = p->bin_orders;
    for (int q = 0; q <= kMaxQ; ++q) {
      int T = p->tile[q] > 0 ? p->tile[q] : 4;
      while (T > 4 && !tile_supported(q, T)) T /= 2;
      bo.tile_of_q[q] = T;
    }
    int32_t* cnt = (int32_t*)(wb + wl.cnt);
    int32_t* fill = (int32_t*)(wb + wl.fill);
    int64_t* start = (int64_t*)(wb + wl.start);
    int64_t* tstart = (int64_t*)(wb + wl.tstart);
    int64_t* ntiles = (int64_t*)(wb + wl.ntiles);
    int64_t* sorted = (int64_t*)(wb + wl.sorted);
    int4* tiles = (int4*)(wb + wl.tiles);
    int64_t* qtile = (int64_t*)(wb + wl.queue);
    unsigned long long* qctr = (unsigned long long*)(wb + wl.queue + 8 * (kNumOrders + 1));
    // captured step: the root passes (which need only the owner map) run on a branch of their
    // own beside the binning and the per-pair target data; the near-edge moments need both
    const bool fork_roots = branches != nullptr && branches->root_fork && branches->root_join;
    hipStream_t rs = fork_roots ? branches->stream[0] : st;
    if (fork_roots && (hipEventRecord(branches->root_fork, st) != hipSuccess ||
                       hipStreamWaitEvent(rs, branches->root_fork, 0) != hipSuccess))
      return RRQ_ERR_DEVICE;
    {
      RootOpts ro;
      for (int q = 0; q <= kMaxQ; ++q) ro.rho_far[q] = p->rho_far[q];
      ro.newton_tol = p->opt.newton_tol;
      ro.newton_maxit = p->opt.newton_maxit;
      double2* root = (double2*)(wb + wl.root);
      uint8_t* nearf = (uint8_t*)(wb + wl.nearf);
      int64_t* nlist = (int64_t*)(wb + wl.nlist);
      double* lamg = (double*)(wb + wl.lamg);
      const int lam_stride = lam_stride_of(p);
      // the Newton and retry lists of the root passes live in the moments' region, which the
      // near-edge moments overwrite only after the root passes (stream order)
      int64_t* qlist = (int64_t*)(wb + wl.lamg);
      int64_t* rlist = qlist + 4 * (tg->nnz > 0 ? tg->nnz : 1);
      if (launch_root(pd, td, owner, ro, (flags & RRQ_F_LEARNED) != 0, root, nearf, qlist,
                      rlist, nlist, counters, pflags, rs) != hipSuccess)
        return RRQ_ERR_DEVICE;
      if (fork_roots && hipEventRecord(branches->root_join, rs) != hipSuccess)
        return RRQ_ERR_DEVICE;
      if (launch_binning(td, p->P, p->order_d, p->perm_d, bo, cnt, fill, start, tstart, ntiles,
                         sorted, tiles, qtile, qctr, st) != hipSuccess)
        return RRQ_ERR_DEVICE;
      double* plocal = (double*)(wb + wl.plocal);
      double* ptd = (double*)(wb + wl.ptd);
      int64_t* pti = (int64_t*)(wb + wl.pti);
      if (launch_pair_local(pd, td, owner, sorted, pot ? nullptr : pair_off, plocal, ptd, pti,
                            st) != hipSuccess)
        return RRQ_ERR_DEVICE;
      ao.ptd = ptd;
      ao.pti = pti;
      if (fork_roots && hipStreamWaitEvent(st, branches->root_join, 0) != hipSuccess)
        return RRQ_ERR_DEVICE;
      for (int qi = 0; qi < kNumOrders; ++qi) {
        const int q = kOrders[qi];
        if (p->patches_h[q].empty()) continue;
        if (launch_lambda(q, pd, p->od[q], td, owner, root, nlist, plocal, counters, pflags, lamg,
                          lam_stride, p->rho_far[q], st) != hipSuccess)
          return RRQ_ERR_DEVICE;
      }
      ao.root = root;
      ao.nearf = nearf;
      ao.lamg = lamg;
      ao.lam_stride = lam_stride;
    }
    // the maps may still be in flight on another stream (captured step)
    if (maps_ready && hipStreamWaitEvent(st, maps_ready, 0) != hipSuccess) return RRQ_ERR_DEVICE;
    if (pot && launch_patch_coef(pd, density, (double*)(wb + wl.pcoef), st) != hipSuccess)
      return RRQ_ERR_DEVICE;
    if (stats && hipEventRecord(ev[0], st) != hipSuccess) return RRQ_ERR_DEVICE;
    // the orders' tile kernels: one after another on the call's stream (timed per order when
    // asked), or, in a captured step with several orders, on branches of their own that fork
    // from and join the call's stream
    int norders = 0;
    for (int qi = 0; qi < kNumOrders; ++qi) norders += !p->patches_h[kOrders[qi]].empty();
    const bool fork = branches != nullptr && norders > 1;
    if (fork && hipEventRecord(branches->fork, st) != hipSuccess) return RRQ_ERR_DEVICE;
    OrderEvents oe;
    for (int qi = 0; qi < kNumOrders; ++qi) {
      const int q = kOrders[qi];
      if (p->patches_h[q].empty()) continue;
      SolveOpts so{p->rho_far[q], p->opt.newton_tol, p->opt.newton_maxit};
      const int T = bo.tile_of_q[q];
      if (!tile_supported(q, T)) return RRQ_ERR_UNSUPPORTED;
      hipStream_t os = st;
      if (fork) {
        os = branches->stream[qi];
        if (hipStreamWaitEvent(os, branches->fork, 0) != hipSuccess) return RRQ_ERR_DEVICE;
      }
      if (order_ms && oe.record(qi, 0, os) != hipSuccess) return RRQ_ERR_DEVICE;
      if (launch_pair_tile(q, T, pot, p->grid[q], pd, p->od[q], td, ao, so, tiles, qtile + qi,
                           qctr + qi * kXcds, sorted, os) != hipSuccess)
        return RRQ_ERR_DEVICE;
      if (order_ms && oe.record(qi, 1, os) != hipSuccess) return RRQ_ERR_DEVICE;
      if (fork && (hipEventRecord(branches->join[qi], os) != hipSuccess ||
                   hipStreamWaitEvent(st, branches->join[qi], 0) != hipSuccess))
        return RRQ_ERR_DEVICE;
    }
    if (order_ms) {
      if (hipStreamSynchronize(st) != hipSuccess) return RRQ_ERR_DEVICE;
      for (int qi = 0; qi < kNumOrders; ++qi) order_ms[qi] = oe.elapsed(qi);
    }
    if (pot && launch_pot_reduce(td, kmask, ao.pairpot, pots, st) != hipSuccess)
      return RRQ_ERR_DEVICE;
  }
  if (stats) {
    unsigned long long h[kNumCounters];
    unsigned hbad = 0;
    float ms = 0.f;
    if (hipEventRecord(ev[1], st) != hipSuccess ||
        hipMemcpyAsync(h, counters, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess || hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess)
      return RRQ_ERR_DEVICE;
    *stats = rrq_stats{};
    stats->kernel_ms = ms;
    stats->pairs = tg->nnz;
    stats->invalid = hbad;
    if (hbad & (kBadNear | kBadSelf | kBadTarget)) return RRQ_ERR_ARG;
    if (hbad & kBadOffsets) return RRQ_ERR_BUFFER;
    stats->near_edges = (int64_t)h[kCNear];
    stats->newton_iters = (int64_t)h[kCIters];
    stats->newton_fail = (int64_t)h[kCFail];
    stats->learned_accept = (int64_t)h[kCLearn];
    stats->newton_max = (int64_t)h[kCMax];
    stats->newton_wave_iters = (int64_t)h[kCWaveIters];
    stats->panel_overflow = (int64_t)h[kCOverflow];
    stats->nonfinite = (int64_t)h[kCNonfinite];
    stats->flagged_pairs = (int64_t)h[kCFlagged];
    for (int qi = 0; qi < kNumOrders; ++qi) stats->order_kernel_ms[qi] = order_ms ? order_ms[qi] : 0.0;
    stats->newton_slots = (int64_t)h[kCNewtonSlots];
    for (int j = 0; j < 5; ++j) stats->newton_over[j] = (int64_t)h[kCNewtonOver + j];
    if (h[kCNonfinite]) return RRQ_ERR_NONFINITE;
  }
  return RRQ_OK;
}

rrq_status rrq_assemble(const rrq_plan* p, const rrq_targets* tg, uint32_t kmask,
                        uint32_t flags, double* out_S, double* out_D, double* out_Sp,
                        double* out_Dp, int64_t out_len, const int64_t* pair_off,
                        uint32_t* pair_flags, void* workspace, size_t workspace_bytes,
                        void* stream, rrq_stats* stats) {
  rrq_status c = check_targets(p, tg);
  if (c != RRQ_OK) return c;
  if (!pair_off || !workspace || (kmask & ~15u) || kmask == 0 || out_len < 0)
    return RRQ_ERR_ARG;
  if (workspace_bytes < ws_bytes(p, tg->nnz)) return RRQ_ERR_BUFFER;
  double* outs[4] = {out_S, out_D, out_Sp, out_Dp};
  for (int K = 0; K < 4; ++K)
    if ((kmask & (1u << K)) && !outs[K]) return RRQ_ERR_ARG;
  if (flags & RRQ_F_LEARNED) {
    if (flags & RRQ_F_PLAIN) return RRQ_ERR_UNSUPPORTED;
    if (!p->has_mlp) return RRQ_ERR_ARG;
  }
  return run_pairs(p, tg, kmask, flags, outs, out_len, pair_off, nullptr, nullptr, pair_flags,
                   workspace, (hipStream_t)stream, stats);
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// allocation-free assembly: the workspace of rrq_assemble taken from a file-scope device
// array instead of a caller buffer
// ---------------------------------------------------------------------------------------
#include <mutex>

static __device__ __align__(256) unsigned char scratch[RRQ_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.  In host
// code the array's name is only a host-side stand-in; kernels must get this address.
rrq_status scratch_for_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return RRQ_ERR_DEVICE;
  if (dev >= kMaxDevices) return RRQ_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
      return RRQ_ERR_DEVICE;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return RRQ_OK;
}
}  // namespace

extern "C" {

rrq_status rrq_assemble_noalloc(const rrq_plan* p, const rrq_targets* tg, uint32_t kmask,
                                uint32_t flags, double* out_S, double* out_D, double* out_Sp,
                                double* out_Dp, int64_t out_len, const int64_t* pair_off,
                                uint32_t* pair_flags, void* stream) {
  rrq_status c = check_targets(p, tg);
  if (c != RRQ_OK) return c;
  if (!pair_off || (kmask & ~15u) || kmask == 0 || out_len < 0) return RRQ_ERR_ARG;
  if (ws_bytes(p, tg->nnz) > (size_t)RRQ_NOALLOC_SCRATCH_BYTES) return RRQ_ERR_BUFFER;
  double* outs[4] = {out_S, out_D, out_Sp, out_Dp};
  for (int K = 0; K < 4; ++K)
    if ((kmask & (1u << K)) && !outs[K]) return RRQ_ERR_ARG;
  if (flags & RRQ_F_LEARNED) {
    if (flags & RRQ_F_PLAIN) return RRQ_ERR_UNSUPPORTED;
    if (!p->has_mlp) return RRQ_ERR_ARG;
  }
  void* ws = nullptr;
  c = scratch_for_current_device(&ws);
  if (c != RRQ_OK) return c;
  // every part of the workspace that must start at zero (counters, bins, queues) is cleared
  // by the kernels of the assembly itself, so the previous call's contents do not matter
  return run_pairs(p, tg, kmask, flags, outs, out_len, pair_off, nullptr, nullptr, pair_flags,
                   ws, (hipStream_t)stream, nullptr);
}

rrq_status rrq_potentials(const rrq_plan* p, const rrq_targets* tg, uint32_t kmask,
                          uint32_t flags, const double* density, double* pot_S, double* pot_D,
                          double* pot_Sp, double* pot_Dp, uint32_t* pair_flags,
                          void* workspace, size_t workspace_bytes, void* stream,
                          rrq_stats* stats) {
  rrq_status c = check_targets(p, tg);
  if (c != RRQ_OK) return c;
  if (!density || !workspace || (kmask & ~15u) || kmask == 0) return RRQ_ERR_ARG;
  if (workspace_bytes < ws_bytes(p, tg->nnz)) return RRQ_ERR_BUFFER;
  double* pots[4] = {pot_S, pot_D, pot_Sp, pot_Dp};
  for (int K = 0; K < 4; ++K)
    if ((kmask & (1u << K)) && !pots[K]) return RRQ_ERR_ARG;
  if (flags & RRQ_F_PLAIN) return RRQ_ERR_UNSUPPORTED;
  if ((flags & RRQ_F_LEARNED) && !p->has_mlp) return RRQ_ERR_ARG;
  return run_pairs(p, tg, kmask, flags, nullptr, 0, nullptr, density, pots, pair_flags,
                   workspace, (hipStream_t)stream, stats);
}

rrq_status rrq_smooth_potentials(const rrq_plan* p, const rrq_targets* tg, uint32_t kmask,
                                 const double* density, double* pot_S, double* pot_D,
                                 double* pot_Sp, double* pot_Dp, void* stream) {
  rrq_status c = check_targets(p, tg);
  if (c != RRQ_OK) return c;
  if (!density || (kmask & ~15u) || kmask == 0) return RRQ_ERR_ARG;
  double* pots[4] = {pot_S, pot_D, pot_Sp, pot_Dp};
  for (int K = 0; K < 4; ++K)
    if ((kmask & (1u << K)) && !pots[K]) return RRQ_ERR_ARG;
  return launch_smooth_direct(p->dev(), tdev(tg), kmask, density, pots, (hipStream_t)stream) ==
                 hipSuccess
             ? RRQ_OK
             : RRQ_ERR_DEVICE;
}

rrq_status rrq_apply(const rrq_plan* p, const rrq_targets* tg, uint32_t kmask,
                     const double* w_S, const double* w_D, const double* w_Sp,
                     const double* w_Dp, const int64_t* pair_off, const double* density,
                     double* pot_S, double* pot_D, double* pot_Sp, double* pot_Dp,
                     void* stream) {
  rrq_status c = check_targets(p, tg);
  if (c != RRQ_OK) return c;
  if (!pair_off || !density || (kmask & ~15u)) return RRQ_ERR_ARG;
  const double* w[4] = {w_S, w_D, w_Sp, w_Dp};
  double* pot[4] = {pot_S, pot_D, pot_Sp, pot_Dp};
  for (int K = 0; K < 4; ++K)
    if ((kmask & (1u << K)) && (!w[K] || !pot[K])) return RRQ_ERR_ARG;
  if (launch_apply(p->dev(), tdev(tg), w, kmask, pair_off, nullptr, density, pot,
                   (hipStream_t)stream) != hipSuccess)
    return RRQ_ERR_DEVICE;
  return RRQ_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// learned initial guess
// ---------------------------------------------------------------------------------------
template <typename T>
static bool talloc(std::vector<void*>& keep, T** p, size_t n) {
  if (dalloc(p, n) != hipSuccess) return false;
  keep.push_back((void*)*p);
  return true;
}
static void tfree(std::vector<void*>& keep) {
  for (void* q : keep) (void)hipFree(q);
  keep.clear();
}

extern "C" rrq_status rrq_collect_roots(const rrq_plan* p, const rrq_targets* tg, int64_t cap,
                                        float* feat, float* dt, double* t0, int64_t* count,
                                        void* stream) {
  rrq_status c = check_targets(p, tg);
  if (c != RRQ_OK) return c;
  if (!count || cap < 0 || (cap > 0 && (!feat || !dt))) return RRQ_ERR_ARG;
  *count = 0;
  if (tg->nnz == 0) return RRQ_OK;
  hipStream_t st = (hipStream_t)stream;
  const int64_t nslot = 4 * tg->nnz;
  std::vector<void*> keep;
  int64_t *owner = nullptr, *flag = nullptr, *part = nullptr;
  unsigned long long* counters = nullptr;
  unsigned* bad = nullptr;
  if (!talloc(keep, &owner, tg->nnz) || !talloc(keep, &counters, kNumCounters) ||
      !talloc(keep, &flag, nslot + 1) || !talloc(keep, &part, scan_partials(nslot)) ||
      !talloc(keep, &bad, 1)) {
    tfree(keep);
    return RRQ_ERR_OOM;
  }
  CollectOpts co;
  for (int q = 0; q <= kMaxQ; ++q) co.rho_far[q] = p->rho_far[q];
  co.newton_tol = p->opt.newton_tol;
  co.newton_maxit = p->opt.newton_maxit;
  const PlanDev pd = p->dev();
  const TargetsDev td = tdev(tg, bad);
  int64_t total = 0;
  unsigned hbad = 0;
  bool ok = launch_validate(pd, td, nullptr, 0, bad, counters, st) == hipSuccess &&
            hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, st) == hipSuccess &&
            hipStreamSynchronize(st) == hipSuccess;
  if (ok && hbad) {
    tfree(keep);
    return RRQ_ERR_ARG;
  }
  ok = ok && launch_owner(td, owner, nullptr, st) == hipSuccess &&
            hipMemsetAsync(flag, 0, 8, st) == hipSuccess &&
            launch_collect(pd, td, owner, co, 0, flag, cap, feat, dt, t0, st) == hipSuccess &&
            launch_scan_i64(flag, nslot, part, st) == hipSuccess &&
            launch_collect(pd, td, owner, co, 1, flag, cap, feat, dt, t0, st) == hipSuccess &&
            hipMemcpyAsync(&total, flag + nslot, 8, hipMemcpyDeviceToHost, st) == hipSuccess &&
            hipStreamSynchronize(st) == hipSuccess;
  tfree(keep);
  if (!ok) return RRQ_ERR_DEVICE;
  *count = total < cap ? total : cap;
  return RRQ_OK;
}

static bool mlp_scratch(std::vector<void*>& keep, MlpScratch& s, int B) {
  return talloc(keep, &s.part, (size_t)kMlpMomBlocks * 20) && talloc(keep, &s.stats, 20) &&
         talloc(keep, &s.p, RRQ_MLP_PARAMS) && talloc(keep, &s.mo, 2 * RRQ_MLP_PARAMS) &&
         talloc(keep, &s.g, RRQ_MLP_PARAMS) && talloc(keep, &s.Xn, (size_t)B * 8) &&
         talloc(keep, &s.H1, (size_t)B * 64) && talloc(keep, &s.H2, (size_t)B * 64) &&
         talloc(keep, &s.dY, (size_t)B * 2) && talloc(keep, &s.dH1, (size_t)B * 64) &&
         talloc(keep, &s.dH2, (size_t)B * 64) && talloc(keep, &s.lossb, (size_t)B);
}

extern "C" rrq_status rrq_mlp_train(const float* feat, const float* dt, int64_t m,
                                    const rrq_mlp_cfg* cfg, float* params, float* loss_curve,
                                    void* stream) {
  if (!feat || !dt || !cfg || !params || m < 1 || cfg->steps < 1 || cfg->batch < 1 ||
      cfg->batch > 65536 || !(cfg->lr > 0.0f))
    return RRQ_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  std::vector<void*> keep;
  MlpScratch s;
  if (!mlp_scratch(keep, s, cfg->batch)) {
    tfree(keep);
    return RRQ_ERR_OOM;
  }
  const bool ok = mlp_train_run(feat, dt, m, cfg->steps, cfg->batch, cfg->lr,
                                (uint64_t)cfg->seed, params, loss_curve, s, st) == hipSuccess &&
                  hipStreamSynchronize(st) == hipSuccess;
  tfree(keep);
  return ok ? RRQ_OK : RRQ_ERR_DEVICE;
}

extern "C" rrq_status rrq_mlp_loss_grad(const float* params, const float* feat, const float* dt,
                                        int64_t n, float* loss, float* grad, void* stream) {
  if (!params || !feat || !dt || !loss || !grad || n < 1 || n > 65536) return RRQ_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  std::vector<void*> keep;
  MlpScratch s;
  if (!mlp_scratch(keep, s, (int)n)) {
    tfree(keep);
    return RRQ_ERR_OOM;
  }
  const bool ok = mlp_loss_grad_run(params, feat, dt, n, loss, grad, s, st) == hipSuccess &&
                  hipStreamSynchronize(st) == hipSuccess;
  tfree(keep);
  return ok ? RRQ_OK : RRQ_ERR_DEVICE;
}

extern "C" rrq_status rrq_mlp_predict(const float* params, const float* feat, int64_t n,
                                      float* out, void* stream) {
  if (!params || n < 0 || (n > 0 && (!feat || !out))) return RRQ_ERR_ARG;
  return mlp_predict_run(params, feat, n, out, (hipStream_t)stream) == hipSuccess
             ? RRQ_OK
             : RRQ_ERR_DEVICE;
}

extern "C" rrq_status rrq_plan_set_mlp(rrq_plan* p, const float* params, void* stream) {
  if (!p) return RRQ_ERR_ARG;
  if (!params) {
    p->has_mlp = false;
    return RRQ_OK;
  }
  if (!p->mlp_d && dalloc(&p->mlp_d, RRQ_MLP_PARAMS) != hipSuccess) return RRQ_ERR_OOM;
  if (mlp_pack_run(params, p->mlp_d, (hipStream_t)stream) != hipSuccess) return RRQ_ERR_DEVICE;
  p->has_mlp = true;
  return RRQ_OK;
}

// ---------------------------------------------------------------------------------------
// autotuner and graph capture
// ---------------------------------------------------------------------------------------
#include <stdio.h>
#include <string>

static std::string order_key(const rrq_plan* p) {
  std::string k;
  for (int q = 0; q <= kMaxQ; ++q)
    if (!p->patches_h[q].empty()) k += std::to_string(q) + "x" + std::to_string(p->patches_h[q].size()) + ";";
  return k;
}

extern "C" rrq_status rrq_autotune(rrq_plan* p, const rrq_targets* tg, uint32_t kmask,
                                   uint32_t flags, double* out_S, double* out_D, double* out_Sp,
                                   double* out_Dp, int64_t out_len, const int64_t* pair_off,
                                   void* workspace, size_t workspace_bytes,
                                   const char* cache_path, void* stream,
                                   rrq_tune_result* result) {
  rrq_status c = check_targets(p, tg);
  if (c != RRQ_OK) return c;
  if (!result) return RRQ_ERR_ARG;
  if (!pair_off || !workspace || (kmask & ~15u) || kmask == 0 || out_len < 0) return RRQ_ERR_ARG;
  if (workspace_bytes < ws_bytes(p, tg->nnz)) return RRQ_ERR_BUFFER;
  double* outs[4] = {out_S, out_D, out_Sp, out_Dp};
  for (int K = 0; K < 4; ++K)
    if ((kmask & (1u << K)) && !outs[K]) return RRQ_ERR_ARG;
  *result = rrq_tune_result{};
  const std::string key = order_key(p);
  auto finish = [&](int from_cache) {
    // summary choice: the order with the longest tuned kernel time
    int big = -1;
    double total = 0.0;
    for (int qi = 0; qi < kNumOrders; ++qi) {
      const int q = kOrders[qi];
      if (p->patches_h[q].empty()) continue;
      result->order_tile[qi] = p->tile[q];
      result->order_grid[qi] = p->grid[q];
      total += result->order_ms[qi];
      if (big < 0 || result->order_ms[qi] > result->order_ms[big]) big = qi;
    }
    result->tile_targets = big >= 0 ? p->tile[kOrders[big]] : 4;
    result->grid = big >= 0 ? p->grid[kOrders[big]] : 2048;
    result->best_ms = total;
    result->from_cache = from_cache;
  };
  if (cache_path) {
    FILE* f = fopen(cache_path, "r");
    if (f) {
      char buf[512];
      bool ok = fgets(buf, sizeof buf, f) && std::string(buf) == key + "\n";
      int tq[kMaxQ + 1] = {}, gq[kMaxQ + 1] = {};
      double mq[kNumOrders] = {};
      for (int qi = 0; ok && qi < kNumOrders; ++qi) {
        const int q = kOrders[qi];
        if (p->patches_h[q].empty()) continue;
        int qq = 0, T = 0, G = 0;
        double ms = 0;
        ok = fscanf(f, "%d %d %d %lf", &qq, &T, &G, &ms) == 4 && qq == q && (T == 4 || T == 8) &&
             G > 0 && G <= (1 << 20);
        tq[q] = T;
        gq[q] = G;
        mq[qi] = ms;
      }
      fclose(f);
      if (ok) {
        for (int qi = 0; qi < kNumOrders; ++qi) {
          const int q = kOrders[qi];
          if (p->patches_h[q].empty()) continue;
          p->tile[q] = tq[q];
          p->grid[q] = gq[q];
          result->order_ms[qi] = mq[qi];
        }
        finish(1);
        return RRQ_OK;
      }
    }
  }
  // every (tile, grid) candidate times every order's tile kernel at once (the orders are
  // separate launches), and each order keeps its own fastest candidate
  hipStream_t st = (hipStream_t)stream;
  const int tiles[2] = {4, 8};
  const int grids[4] = {512, 1024, 2048, 4096};
  double best[kNumOrders];
  int bT[kNumOrders], bG[kNumOrders];
  for (int qi = 0; qi < kNumOrders; ++qi) {
    best[qi] = 1e300;
    bT[qi] = p->tile[kOrders[qi]];
    bG[qi] = p->grid[kOrders[qi]];
  }
  flags &= ~(uint32_t)RRQ_F_PLAIN;
  for (int T : tiles)
    for (int G : grids) {
      for (int q = 0; q <= kMaxQ; ++q) {
        p->tile[q] = T;
        p->grid[q] = G;
      }
      float ms[kNumOrders] = {};
      rrq_status r = run_pairs(p, tg, kmask, flags, outs, out_len, pair_off, nullptr, nullptr,
                               nullptr, workspace, st, nullptr);          // warm
      if (r == RRQ_OK)
        r = run_pairs(p, tg, kmask, flags, outs, out_len, pair_off, nullptr, nullptr, nullptr,
                      workspace, st, nullptr, nullptr, nullptr, ms);
      if (r != RRQ_OK) continue;
      for (int qi = 0; qi < kNumOrders; ++qi) {
        const int q = kOrders[qi];
        if (p->patches_h[q].empty()) continue;
        int Te = T;                         // the tile size this order actually ran with
        while (Te > 4 && !tile_supported(q, Te)) Te /= 2;
        if (ms[qi] > 0.f && ms[qi] < best[qi]) {
          best[qi] = ms[qi];
          bT[qi] = Te;
          bG[qi] = G;
        }
      }
    }
  bool any = false;
  for (int qi = 0; qi < kNumOrders; ++qi) {
    const int q = kOrders[qi];
    p->tile[q] = bT[qi];
    p->grid[q] = bG[qi];
    if (!p->patches_h[q].empty()) {
      if (best[qi] >= 1e300) return RRQ_ERR_DEVICE;
      result->order_ms[qi] = best[qi];
      any = true;
    }
  }
  if (!any) return RRQ_ERR_DEVICE;
  finish(0);
  if (cache_path) {
    FILE* f = fopen(cache_path, "w");
    if (f) {
      fprintf(f, "%s\n", key.c_str());
      for (int qi = 0; qi < kNumOrders; ++qi)
        if (!p->patches_h[kOrders[qi]].empty())
          fprintf(f, "%d %d %d %.6f\n", kOrders[qi], bT[qi], bG[qi], best[qi]);
      fclose(f);
    }
  }
  return RRQ_OK;
}

struct rrq_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" rrq_status rrq_graph_create(rrq_plan* p, const rrq_surface* s, const rrq_targets* tg,
                                       uint32_t kmask, uint32_t flags, double* out_S,
                                       double* out_D, double* out_Sp, double* out_Dp,
                                       int64_t out_len, int64_t* pair_off, void* workspace,
                                       size_t workspace_bytes, void* stream, rrq_graph** out) {
  if (!out || !p) return RRQ_ERR_ARG;
  *out = nullptr;
  rrq_status c = check_targets(p, tg);
  if (c != RRQ_OK) return c;
  c = check_surface(s);
  if (c != RRQ_OK) return c;
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return RRQ_ERR_DEVICE;
  // the capture stream starts after the work already queued on the caller's stream
  {
    hipEvent_t after = nullptr;
    const bool ok = hipEventCreateWithFlags(&after, hipEventDisableTiming) == hipSuccess &&
                    hipEventRecord(after, (hipStream_t)stream) == hipSuccess &&
                    hipStreamWaitEvent(cs, after, 0) == hipSuccess;
    if (after) (void)hipEventDestroy(after);
    if (!ok) {
      (void)hipStreamDestroy(cs);
      return RRQ_ERR_DEVICE;
    }
  }
  // one eager pass on the capture stream first: kernel attributes are set outside capture
  rrq_status r = rrq_plan_refit(p, s, cs);
  if (r == RRQ_OK) r = rrq_pair_offsets(p, tg, pair_off, workspace, workspace_bytes, nullptr, cs);
  if (r == RRQ_OK)
    r = rrq_assemble(p, tg, kmask, flags, out_S, out_D, out_Sp, out_Dp, out_len, pair_off,
                     nullptr, workspace, workspace_bytes, cs, nullptr);
  if (r != RRQ_OK || hipStreamSynchronize(cs) != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return r != RRQ_OK ? r : RRQ_ERR_DEVICE;
  }
  rrq_graph* g = new (std::nothrow) rrq_graph();
  if (!g) { (void)hipStreamDestroy(cs); return RRQ_ERR_OOM; }
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    delete g;
    (void)hipStreamDestroy(cs);
    return RRQ_ERR_DEVICE;
  }
  // captured step: geometry, then the fits (maps) on a second stream beside the edge tables,
  // pair offsets, binning and pre-passes; the tile kernels wait for them
  hipStream_t ms = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  bool ok = hipStreamCreateWithFlags(&ms, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&fork, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&join, hipEventDisableTiming) == hipSuccess;
  // branches of the orders' tile kernels
  OrderBranches br{};
  for (int qi = 0; ok && qi < kNumOrders; ++qi)
    ok = hipStreamCreateWithFlags(&br.stream[qi], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&br.join[qi], hipEventDisableTiming) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&br.fork, hipEventDisableTiming) == hipSuccess &&
       hipEventCreateWithFlags(&br.root_fork, hipEventDisableTiming) == hipSuccess &&
       hipEventCreateWithFlags(&br.root_join, hipEventDisableTiming) == hipSuccess;
  r = ok ? run_geometry(p, s, cs) : RRQ_ERR_DEVICE;
  if (r == RRQ_OK && (hipEventRecord(fork, cs) != hipSuccess ||
                      hipStreamWaitEvent(ms, fork, 0) != hipSuccess))
    r = RRQ_ERR_DEVICE;
  // the maps and the edge tables, which only the tile kernels read, on the second branch;
  // the pair offsets, binning, roots and near-edge moments on this one
  if (r == RRQ_OK) r = run_fits(p, ms);
  if (r == RRQ_OK) r = run_edge_tables(p, ms);
  if (r == RRQ_OK && hipEventRecord(join, ms) != hipSuccess) r = RRQ_ERR_DEVICE;
  if (r == RRQ_OK) r = rrq_pair_offsets(p, tg, pair_off, workspace, workspace_bytes, nullptr, cs);
  if (r == RRQ_OK) {
    double* outs[4] = {out_S, out_D, out_Sp, out_Dp};
    r = run_pairs(p, tg, kmask, flags, outs, out_len, pair_off, nullptr, nullptr, nullptr,
                  workspace, cs, nullptr, join, &br);
  }
  hipError_t ec = hipStreamEndCapture(cs, &g->graph);
  if (join) (void)hipEventDestroy(join);
  if (fork) (void)hipEventDestroy(fork);
  if (ms) (void)hipStreamDestroy(ms);
  if (br.fork) (void)hipEventDestroy(br.fork);
  if (br.root_fork) (void)hipEventDestroy(br.root_fork);
  if (br.root_join) (void)hipEventDestroy(br.root_join);
  for (int qi = 0; qi < kNumOrders; ++qi) {
    if (br.join[qi]) (void)hipEventDestroy(br.join[qi]);
    if (br.stream[qi]) (void)hipStreamDestroy(br.stream[qi]);
  }
  if (r == RRQ_OK && ec == hipSuccess &&
      hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) == hipSuccess) {
    (void)hipStreamDestroy(cs);
    *out = g;
    return RRQ_OK;
  }
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  (void)hipStreamDestroy(cs);
  return r != RRQ_OK ? r : RRQ_ERR_DEVICE;
}

extern "C" rrq_status rrq_graph_launch(rrq_graph* g, void* stream) {
  if (!g || !g->exec) return RRQ_ERR_ARG;
  return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? RRQ_OK : RRQ_ERR_DEVICE;
}

extern "C" rrq_status rrq_graph_destroy(rrq_graph* g) {
  if (!g) return RRQ_ERR_ARG;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return RRQ_OK;
}
