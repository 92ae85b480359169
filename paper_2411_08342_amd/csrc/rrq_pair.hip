// Target-dependent steps (Steps 4-8 of the algorithm in Sec. 4) in the plain form: one
// workgroup per (target, patch) near pair.  Also the pair-owner map, the pair offsets and the
// sparse apply.
#include "rrq_device.h"
#include "rrq_internal.h"

namespace rrq {

constexpr int PNT = 256;
// panel capacity per near edge of the plain form: the largest of the batched form's
// per-order capacities (wave_panel_cap), so that both forms keep the same leaves
constexpr int kMaxPanels = 320;

// ---------------------------------------------------------------------------------------
// device check of the caller's targets, near list, self indices and pair offsets.  Bits of
// *bad: kBadNear (row pointer not from 0 to nnz or decreasing, patch index out of range),
// kBadSelf (self_patch outside [-1, P), or self_node outside the self patch's nodes),
// kBadTarget (a target point or normal not finite), kBadOffsets
// (pair_off[0] != 0, a block size other than q_P^2, or pair_off[nnz] > out_len).  Only
// in-range entries are read: near_ptr[0..T], near_patch[0..nnz), self_*[0..T),
// pair_off[0..nnz].
// ---------------------------------------------------------------------------------------
__global__ void k_validate_clear(unsigned* bad, unsigned long long* counters) {
  if (threadIdx.x == 0) *bad = 0u;
  if (counters != nullptr && threadIdx.x < kNumCounters) counters[threadIdx.x] = 0ull;
}

__global__ void k_validate(PlanDev pd, TargetsDev tg, const int64_t* pair_off, int64_t out_len,
                           unsigned* bad) {
  unsigned f = 0u;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t t = gid; t <= tg.T; t += stride) {
    const int64_t a = tg.near_ptr[t];
    if (t == 0 && a != 0) f |= kBadNear;
    if (t == tg.T) {
      if (a != tg.nnz) f |= kBadNear;
    } else {
      if (a > tg.near_ptr[t + 1]) f |= kBadNear;
      for (int c = 0; c < 3; ++c)
        if (!isfinite(tg.xyz[c * tg.T + t]) || !isfinite(tg.nrm[c * tg.T + t])) f |= kBadTarget;
      const int sp = tg.self_patch[t];
      if (sp < -1 || sp >= pd.npatch) {
        f |= kBadSelf;
      } else if (sp >= 0) {
        const int q = pd.order[sp], sn = tg.self_node[t];
        if (sn < 0 || sn >= q * q) f |= kBadSelf;
      }
    }
  }
  for (int64_t k = gid; k < tg.nnz; k += stride) {
    const int P = tg.near_patch[k];
    if (P < 0 || P >= pd.npatch) {
      f |= kBadNear;
    } else if (pair_off != nullptr) {
      const int q = pd.order[P];
      if (pair_off[k + 1] - pair_off[k] != (int64_t)q * q) f |= kBadOffsets;
    }
  }
  if (pair_off != nullptr && gid == 0 && (pair_off[0] != 0 || pair_off[tg.nnz] > out_len))
    f |= kBadOffsets;
  if (f) atomicOr(bad, f);
}

hipError_t launch_validate(const PlanDev& pd, const TargetsDev& tg, const int64_t* pair_off,
                           int64_t out_len, unsigned* bad, unsigned long long* counters,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_validate_clear, dim3(1), dim3(64), 0, st, bad, counters);
  const int64_t n = (tg.T + 1 > tg.nnz ? tg.T + 1 : tg.nnz);
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_validate, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(256), 0, st, pd,
                     tg, pair_off, out_len, bad);
  return hipGetLastError();
}

// owner[k] = target of near pair k; pflags[k] = 0
__global__ void k_owner(TargetsDev tg, int64_t* owner, uint32_t* pflags) {
  if (input_bad(tg)) return;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tg.T;
       t += (int64_t)gridDim.x * blockDim.x)
    for (int64_t k = tg.near_ptr[t]; k < tg.near_ptr[t + 1]; ++k) {
      owner[k] = t;
      if (pflags != nullptr) pflags[k] = 0u;
    }
}

hipError_t launch_owner(const TargetsDev& tg, int64_t* owner, uint32_t* pflags,
                        hipStream_t st) {
  int64_t g = (tg.T + 255) / 256;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_owner, dim3((unsigned)(g < 65535 ? g : 65535)), dim3(256), 0, st, tg,
                     owner, pflags);
  return hipGetLastError();
}

// pair sizes q_P^2, then an inclusive scan
__global__ void k_pair_sizes(PlanDev pd, TargetsDev tg, int64_t* off) {
  if (input_bad(tg)) return;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < tg.nnz;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int q = pd.order[tg.near_patch[k]];
    off[k + 1] = (int64_t)q * q;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) off[0] = 0;
}

// Inclusive scan of a[1..n] in three passes: every workgroup scans a segment of kScanSeg
// elements (8 consecutive per thread) and records the segment total; one workgroup scans
// the totals (exclusive); every segment then adds its prefix.
constexpr int kScanThreads = 1024, kScanPer = 8, kScanSeg = kScanThreads * kScanPer;

int64_t scan_partials(int64_t n) { return (n + kScanSeg - 1) / kScanSeg + 1; }

__device__ __forceinline__ int64_t block_incl_scan(int64_t v, int64_t* sm) {
  const int t = threadIdx.x;
  sm[t] = v;
  __syncthreads();
  for (int o = 1; o < kScanThreads; o <<= 1) {
    const int64_t x = t >= o ? sm[t - o] : 0;
    __syncthreads();
    sm[t] += x;
    __syncthreads();
  }
  return sm[t];
}

__global__ __launch_bounds__(kScanThreads) void k_scan_seg(int64_t* a, int64_t n, int64_t* part) {
  __shared__ int64_t sm[kScanThreads];
  const int64_t base = 1 + (int64_t)blockIdx.x * kScanSeg + (int64_t)threadIdx.x * kScanPer;
  int64_t v[kScanPer];
  int64_t sum = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    const int64_t idx = base + i;
    sum += idx <= n ? a[idx] : 0;
    v[i] = sum;
  }
  const int64_t incl = block_incl_scan(sum, sm);
  const int64_t excl = incl - sum;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    const int64_t idx = base + i;
    if (idx <= n) a[idx] = v[i] + excl;
  }
  if (threadIdx.x == kScanThreads - 1) part[blockIdx.x] = incl;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_part(int64_t* part, int64_t nseg) {
  __shared__ int64_t sm[kScanThreads];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t b = 0; b < nseg; b += kScanThreads) {
    const int64_t i = b + threadIdx.x;
    const int64_t v = i < nseg ? part[i] : 0;
    const int64_t incl = block_incl_scan(v, sm);
    const int64_t c = carry;
    if (i < nseg) part[i] = c + incl - v;       // exclusive
    __syncthreads();
    if (threadIdx.x == kScanThreads - 1) carry = c + incl;
    __syncthreads();
  }
}

__global__ void k_scan_add(int64_t* a, int64_t n, const int64_t* part) {
  const int64_t seg = blockIdx.x + 1;           // segment 0 has prefix 0
  const int64_t add = part[seg];
  const int64_t base = 1 + seg * kScanSeg;
  for (int64_t i = base + threadIdx.x; i < base + kScanSeg && i <= n; i += blockDim.x) a[i] += add;
}

hipError_t launch_scan_i64(int64_t* a, int64_t n, int64_t* part, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t nseg = (n + kScanSeg - 1) / kScanSeg;
  hipLaunchKernelGGL(k_scan_seg, dim3((unsigned)nseg), dim3(kScanThreads), 0, st, a, n, part);
  hipLaunchKernelGGL(k_scan_part, dim3(1), dim3(kScanThreads), 0, st, part, nseg);
  if (nseg > 1)
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)(nseg - 1)), dim3(256), 0, st, a, n, part);
  return hipGetLastError();
}

hipError_t launch_pair_offsets(const PlanDev& pd, const TargetsDev& tg, int64_t* pair_off,
                               int64_t* part, hipStream_t st) {
  int64_t g = (tg.nnz + 255) / 256;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_pair_sizes, dim3((unsigned)(g < 65535 ? g : 65535)), dim3(256), 0, st,
                     pd, tg, pair_off);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_scan_i64(pair_off, tg.nnz, part, st);
}

// ---------------------------------------------------------------------------------------
// shared-memory state of one pair
// ---------------------------------------------------------------------------------------
template <int Q>
struct PairSmem {
  static constexpr int PT = 2 * Q, NP = np_of(Q), NJK = njk_of(Q);
  double fr[kFrame];
  double x[3], nu[3], u[3];
  double eloc[4 * PT * 3], etan[4 * PT * 3], ecoef[4 * PT * 3];
  double t0[4][2];
  int near[4];
  int npan[4];
  double lam1[4][PT], lam3[4][PT];
  double pt_tau[PNT], pt_w1[PNT], pt_w3[PNT];
  int pt_hit[PNT];
  double w1[4 * PT], w3[4 * PT], d[4 * PT * 3], av[4 * PT * 3];
  double pan[4][kMaxPanels][2];
  cplx V[NJK];
  cplx Qv[NJK][4];
  cplx dQ[NJK][4];
  double Om[4], dOm[4];     // (Omega_0, Omega_vec) and d/dnu'
  cplx Rt[tri(Q, Q) + 1];   // target solid harmonics table at permuted point
  cplx gSnu[tri(Q, Q) + 1]; // grad S^{ab}(x) . nu'
  double rD[4 * NP], rSp[4 * NP], rS[5 * NP], rDp[4 * NP];
  double red[PNT / 64];
  double cand_d[PNT / 64];
  int cand_i[PNT / 64];
};

template <int Q>
__global__ __launch_bounds__(PNT) void k_pair_plain(PlanDev pd, OrderDev od, TargetsDev tg,
                                                    AssembleOut out, SolveOpts so) {
  constexpr int PT = 2 * Q, NP = np_of(Q), NJK = njk_of(Q), Q2 = Q * Q;
  __shared__ PairSmem<Q> S;
  const int tid = threadIdx.x;
  if (input_bad(tg)) return;
  for (int64_t k = blockIdx.x; k < tg.nnz; k += gridDim.x) {
    const int P = tg.near_patch[k];
    if (pd.order[P] != Q) continue;
    const int64_t t = out.owner[k];
    const int self = (tg.self_patch[t] == P) ? tg.self_node[t] : -1;
    const int64_t n0 = pd.node_off[P];
    const int64_t e0 = pd.edge_off[P];
    __syncthreads();
    if (tid < kFrame) S.fr[tid] = pd.frame[(int64_t)P * kFrame + tid];
    for (int i = tid; i < 4 * PT * 3; i += PNT) {
      const int c = i % 3, ei = i / 3;
      S.eloc[i] = pd.edge_loc[c * pd.E + e0 + ei];
      S.etan[i] = pd.edge_tan[c * pd.E + e0 + ei];
      S.ecoef[i] = pd.edge_coef[c * pd.E + e0 + ei];
    }
    __syncthreads();
    // target in local coordinates
    if (tid == 0) {
      const double inv_s = 1.0 / S.fr[12];
      double dx[3], nv[3];
      for (int c = 0; c < 3; ++c) {
        dx[c] = tg.xyz[c * tg.T + t] - S.fr[c];
        nv[c] = tg.nrm[c * tg.T + t];
      }
      for (int a = 0; a < 3; ++a) {
        const double* ax = S.fr + 3 + 3 * a;
        S.x[a] = (dx[0] * ax[0] + dx[1] * ax[1] + dx[2] * ax[2]) * inv_s;
        S.nu[a] = nv[0] * ax[0] + nv[1] * ax[1] + nv[2] * ax[2];
      }
    }
    __syncthreads();
    // u: nu' for a self target, else +-nu of the nearest node (lowest index on ties)
    if (self >= 0) {
      if (tid < 3) S.u[tid] = S.nu[tid];
    } else {
      // bi starts at a valid node, so that non-finite distances still select a node
      double bd = 1e300;
      int bi = 0;
      for (int i = tid; i < Q2; i += PNT) {
        double d2 = 0;
        for (int c = 0; c < 3; ++c) {
          const double dd = S.x[c] - pd.node_loc[c * pd.N + n0 + i];
          d2 += dd * dd;
        }
        if (d2 < bd || (d2 == bd && i < bi)) { bd = d2; bi = i; }
      }
      for (int o = 32; o > 0; o >>= 1) {
        double od2 = __shfl_xor(bd, o, 64);
        int oi = __shfl_xor(bi, o, 64);
        if (od2 < bd || (od2 == bd && oi < bi)) { bd = od2; bi = oi; }
      }
      if ((tid & 63) == 0) { S.cand_d[tid >> 6] = bd; S.cand_i[tid >> 6] = bi; }
      __syncthreads();
      if (tid == 0) {
        for (int w = 1; w < PNT / 64; ++w)
          if (S.cand_d[w] < bd || (S.cand_d[w] == bd && S.cand_i[w] < bi)) {
            bd = S.cand_d[w];
            bi = S.cand_i[w];
          }
        double nv[3], dd = 0;
        for (int c = 0; c < 3; ++c) {
          nv[c] = pd.node_loc[(3 + c) * pd.N + n0 + bi];
          dd += (S.x[c] - pd.node_loc[c * pd.N + n0 + bi]) * nv[c];
        }
        const double sg = dd >= 0.0 ? 1.0 : -1.0;
        for (int c = 0; c < 3; ++c) S.u[c] = sg * nv[c];
      }
    }
    __syncthreads();
    // Step 5 per edge: classification, Newton root, moments
    if (tid < 4) {
      const int e = tid;
      const double* cf = S.ecoef + e * PT * 3;
      // end points r(-1) = sum_k (-1)^k c_k, r(1) = sum_k c_k (P_k(+-1) = (+-1)^k)
      double A[3] = {0, 0, 0}, B[3] = {0, 0, 0};
      for (int kk = 0; kk < PT; ++kk)
        for (int c = 0; c < 3; ++c) {
          A[c] += (kk & 1) ? -cf[kk * 3 + c] : cf[kk * 3 + c];
          B[c] += cf[kk * 3 + c];
        }
      double m[3], dv[3], v[3];
      for (int c = 0; c < 3; ++c) {
        m[c] = 0.5 * (A[c] + B[c]);
        dv[c] = 0.5 * (B[c] - A[c]);
        v[c] = S.x[c] - m[c];
      }
      const double dd = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
      const double cr0 = dv[1] * v[2] - dv[2] * v[1];
      const double cr1 = dv[2] * v[0] - dv[0] * v[2];
      const double cr2 = dv[0] * v[1] - dv[1] * v[0];
      cplx ts = mk((dv[0] * v[0] + dv[1] * v[1] + dv[2] * v[2]) / dd,
                   sqrt(cr0 * cr0 + cr1 * cr1 + cr2 * cr2) / dd);
      int near = 0, its = 0, conv = 1;
      cplx t0 = ts;
      if (bernstein_rho(ts) <= so.rho_far) {
        conv = 0;
        for (its = 1; its <= so.newton_maxit; ++its) {
          cplx r[3], dr[3];
          leg3(cf, 3, PT, t0, r, dr);
          cplx f = mk(0, 0), fp = mk(0, 0);
          for (int c = 0; c < 3; ++c) {
            cplx ec = r[c] - mk(S.x[c], 0.0);
            f = f + ec * ec;
            fp = fp + ec * dr[c];
          }
          fp = 2.0 * fp;
          cplx dt = cdiv(f, fp);
          t0 = t0 - dt;
          if (cabsd(dt) <= so.newton_tol * fmax(1.0, cabsd(t0))) { conv = 1; break; }
        }
        if (its > so.newton_maxit) its = so.newton_maxit;
        if (t0.im < 0) t0.im = -t0.im;
        if (conv && bernstein_rho(t0) <= so.rho_far) near = 1;
        atomicAdd(&out.counters[kCIters], (unsigned long long)its);
        if (!conv) {
          atomicAdd(&out.counters[kCFail], 1ull);
          flag_pair(out.pflags, out.counters, k, kFlagNewton);
        }
        atomicMax(&out.counters[kCMax], (unsigned long long)its);
      }
      S.near[e] = near;
      S.t0[e][0] = t0.re;
      S.t0[e][1] = t0.im;
      if (near) {
        atomicAdd(&out.counters[kCNear], 1ull);
        // graded panels: dyadic bisection toward Re t0 until every panel sees t0 at
        // Bernstein radius >= rho_far in its own scaled coordinate
        double stk[64][3];
        int sp = 0, np_ = 0;
        stk[sp][0] = -1.0; stk[sp][1] = 1.0; stk[sp][2] = 0; ++sp;
        while (sp > 0) {
          --sp;
          const double lo = stk[sp][0], hi = stk[sp][1];
          const int lev = (int)stk[sp][2];
          const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
          const double rho = bernstein_rho(mk((t0.re - c) / h, t0.im / h));
          if (lev >= 60 || rho >= so.rho_far || sp >= 62) {
            if (np_ < kMaxPanels) {
              S.pan[e][np_][0] = lo;
              S.pan[e][np_][1] = hi;
              ++np_;
            } else {
              atomicAdd(&out.counters[kCOverflow], 1ull);
              flag_pair(out.pflags, out.counters, k, kFlagPanels);
            }
          } else {
            stk[sp][0] = c; stk[sp][1] = hi; stk[sp][2] = lev + 1; ++sp;
            stk[sp][0] = lo; stk[sp][1] = c; stk[sp][2] = lev + 1; ++sp;
          }
        }
        S.npan[e] = np_;
      } else {
        S.npan[e] = 0;
      }
    }
    __syncthreads();
    // Lagrange-basis moments of near edges, lambda_i^{(m)} = int l_i(t) |t - t0|^{-m} dt
    // (the vector U^T I^{(m)} of the singularity swap), by GL quadrature on the graded panels
    // with barycentric l_i; Omega_0 of near edges on the same points.
    double om_near = 0.0;
    for (int e = 0; e < 4; ++e) {
      if (!S.near[e]) continue;
      const int npts = S.npan[e] * PT;
      const double a = S.t0[e][0], b = S.t0[e][1];
      double l1 = 0.0, l3 = 0.0;
      for (int base = 0; base < npts; base += PNT) {
        const int idx = base + tid;
        if (idx < npts) {
          const int pn = idx / PT, g = idx % PT;
          const double lo = S.pan[e][pn][0], hi = S.pan[e][pn][1];
          const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
          const double tau = c + h * od.gl_t[g];
          const double K2 = (tau - a) * (tau - a) + b * b;
          const double K1 = 1.0 / sqrt(K2);
          const double hw = h * od.gl_w[g];
          double den = 0.0;
          int hit = -1;
          for (int j = 0; j < PT; ++j) {
            const double dt = tau - od.gl_t[j];
            if (dt == 0.0) hit = j;
            else den += od.bary[j] / dt;
          }
          const double sc1 = hit >= 0 ? hw * K1 : hw * K1 / den;
          S.pt_tau[tid] = tau;
          S.pt_w1[tid] = sc1;
          S.pt_w3[tid] = sc1 / K2;
          S.pt_hit[tid] = hit;
          cplx r[3], dr[3];
          leg3(S.ecoef + e * PT * 3, 3, PT, mk(tau, 0.0), r, dr);
          const double rr[3] = {r[0].re, r[1].re, r[2].re};
          const double dd[3] = {dr[0].re, dr[1].re, dr[2].re};
          om_near += hw * omega0_at(S.x, S.u, rr, dd);
        } else {
          S.pt_tau[tid] = 3.0;
          S.pt_w1[tid] = 0.0;
          S.pt_w3[tid] = 0.0;
          S.pt_hit[tid] = -2;
        }
        __syncthreads();
        if (tid < PT) {
          const int cnt = npts - base < PNT ? npts - base : PNT;
          const double ti = od.gl_t[tid], bi = od.bary[tid];
          for (int pidx = 0; pidx < cnt; ++pidx) {
            const int hit = S.pt_hit[pidx];
            double li;
            if (hit >= 0) li = hit == tid ? 1.0 : 0.0;
            else li = bi / (S.pt_tau[pidx] - ti);
            l1 += S.pt_w1[pidx] * li;
            l3 += S.pt_w3[pidx] * li;
          }
        }
        __syncthreads();
      }
      if (tid < PT) {
        S.lam1[e][tid] = l1;
        S.lam3[e][tid] = l3;
      }
    }
    __syncthreads();
    // effective weights per (edge, node)
    double om_far = 0, ov0 = 0, ov1 = 0, ov2 = 0, dv0 = 0, dv1 = 0, dv2 = 0, dom0 = 0;
    for (int idx = tid; idx < 4 * PT; idx += PNT) {
      const int e = idx / PT, i = idx % PT;
      double d[3];
      for (int c = 0; c < 3; ++c) d[c] = S.x[c] - S.eloc[idx * 3 + c];
      const double R2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      const double R = sqrt(R2);
      double w1, w3;
      if (S.near[e]) {
        const double l1 = S.lam1[e][i], l3 = S.lam3[e][i];
        const double ta = od.gl_t[i] - S.t0[e][0], tb = S.t0[e][1];
        const double tt = sqrt(ta * ta + tb * tb);
        const double q1 = tt / R;
        w1 = l1 * q1;
        w3 = l3 * q1 * q1 * q1;
      } else {
        w1 = od.gl_w[i] / R;
        w3 = od.gl_w[i] / (R2 * R);
        om_far += od.gl_w[i] * omega0_at(S.x, S.u, S.eloc + idx * 3, S.etan + idx * 3);
      }
      const double dn = d[0] * S.nu[0] + d[1] * S.nu[1] + d[2] * S.nu[2];
      S.w1[idx] = w1;
      S.w3[idx] = w3;
      for (int c = 0; c < 3; ++c) {
        S.d[idx * 3 + c] = d[c];
        S.av[idx * 3 + c] = w1 * S.nu[c] - w3 * dn * d[c];
      }
      const double* rp = S.etan + idx * 3;
      ov0 -= w1 * rp[0];
      ov1 -= w1 * rp[1];
      ov2 -= w1 * rp[2];
      dv0 += w3 * dn * rp[0];
      dv1 += w3 * dn * rp[1];
      dv2 += w3 * dn * rp[2];
      // grad Omega_0 . nu' = -sum w3 (r' x d) . nu'
      const double cx = rp[1] * d[2] - rp[2] * d[1];
      const double cy = rp[2] * d[0] - rp[0] * d[2];
      const double cz = rp[0] * d[1] - rp[1] * d[0];
      dom0 -= w3 * (cx * S.nu[0] + cy * S.nu[1] + cz * S.nu[2]);
    }
    om_far += om_near;
    {
      double v;
      v = block_sum<PNT>(om_far, S.red); if (tid == 0) S.Om[0] = v;
      v = block_sum<PNT>(ov0, S.red); if (tid == 0) S.Om[1] = v;
      v = block_sum<PNT>(ov1, S.red); if (tid == 0) S.Om[2] = v;
      v = block_sum<PNT>(ov2, S.red); if (tid == 0) S.Om[3] = v;
      v = block_sum<PNT>(dom0, S.red); if (tid == 0) S.dOm[0] = v;
      v = block_sum<PNT>(dv0, S.red); if (tid == 0) S.dOm[1] = v;
      v = block_sum<PNT>(dv1, S.red); if (tid == 0) S.dOm[2] = v;
      v = block_sum<PNT>(dv2, S.red); if (tid == 0) S.dOm[3] = v;
    }
    __syncthreads();
    // Step 6: line integrals V^{jk}, Q^{jk}, dQ^{jk} (thread per (j,k)); Step 4: target table
    if (tid < NJK) {
      const int n = tid;
      const double* tb = pd.tabs + pd.tab_off[P];
      cplx V = mk(0, 0), Qs = mk(0, 0), Q1 = mk(0, 0), Q2_ = mk(0, 0), Q3 = mk(0, 0);
      cplx Ds = mk(0, 0), D1 = mk(0, 0), D2 = mk(0, 0), D3 = mk(0, 0);
      for (int e = 0; e < 4; ++e)
        for (int i = 0; i < PT; ++i) {
          const int idx = e * PT + i;
          const double2* o = (const double2*)tb + (int64_t)idx * 6 * NJK + n;
          const cplx c0 = mk(o[0].x, o[0].y), c1 = mk(o[NJK].x, o[NJK].y);
          const cplx c2 = mk(o[2 * NJK].x, o[2 * NJK].y), h0 = mk(o[3 * NJK].x, o[3 * NJK].y);
          const cplx h1 = mk(o[4 * NJK].x, o[4 * NJK].y), h2 = mk(o[5 * NJK].x, o[5 * NJK].y);
          const double w1 = S.w1[idx];
          const double d0 = S.d[idx * 3], d1 = S.d[idx * 3 + 1], d2 = S.d[idx * 3 + 2];
          V = V + w1 * (d0 * c0 + d1 * c1 + d2 * c2);
          // (0, v)(0, h) = (-v.h, v x h)
          const double v0 = w1 * d0, v1 = w1 * d1, v2 = w1 * d2;
          Qs = Qs - (v0 * h0 + v1 * h1 + v2 * h2);
          Q1 = Q1 + (v1 * h2 - v2 * h1);
          Q2_ = Q2_ + (v2 * h0 - v0 * h2);
          Q3 = Q3 + (v0 * h1 - v1 * h0);
          const double a0 = S.av[idx * 3], a1 = S.av[idx * 3 + 1], a2 = S.av[idx * 3 + 2];
          Ds = Ds - (a0 * h0 + a1 * h1 + a2 * h2);
          D1 = D1 + (a1 * h2 - a2 * h1);
          D2 = D2 + (a2 * h0 - a0 * h2);
          D3 = D3 + (a0 * h1 - a1 * h0);
        }
      S.V[n] = V;
      S.Qv[n][0] = Qs; S.Qv[n][1] = Q1; S.Qv[n][2] = Q2_; S.Qv[n][3] = Q3;
      S.dQ[n][0] = Ds; S.dQ[n][1] = D1; S.dQ[n][2] = D2; S.dQ[n][3] = D3;
    }
    if (tid == PNT - 1) solid_table<Q>(S.x[1], S.x[2], S.x[0], S.Rt);
    __syncthreads();
    for (int idx = tid; idx < tri(Q, Q) + 1; idx += PNT) {
      int a = 0;
      while (tri(a + 1, 0) <= idx) ++a;
      const int b = idx - tri(a, 0);
      cplx acc = mk(0, 0);
      for (int c = 0; c < 3; ++c) acc = acc + S.nu[c] * dS(S.Rt, a, b, c);
      S.gSnu[idx] = acc;
    }
    __syncthreads();
    // Steps 7-8: translation and moments, thread per basis function (l, m)
    if (tid < NP) {
      const int lm = tid;
      int l = 1;
      while (np_of(l) <= lm) ++l;
      const int m = lm - np_of(l - 1) + 1;
      cplx Ia[4] = {mk(0, 0), mk(0, 0), mk(0, 0), mk(0, 0)};
      cplx dIa[4] = {mk(0, 0), mk(0, 0), mk(0, 0), mk(0, 0)};
      for (int it = od.dlp_ptr[lm]; it < od.dlp_ptr[lm + 1]; ++it) {
        const Term tm = od.dlp[it];
        const cplx s_ = rget(S.Rt, tm.a, tm.b);
        cplx gs;
        if (tm.b >= 0) gs = S.gSnu[tri(tm.a, tm.b)];
        else {
          cplx g = S.gSnu[tri(tm.a, -tm.b)];
          gs = ((-tm.b) & 1) ? mk(-g.re, g.im) : mk(g.re, -g.im);
        }
        for (int c = 0; c < 4; ++c) {
          cplx X = S.Qv[tm.n][c], dX = S.dQ[tm.n][c];
          if (tm.neg) { X = conjg(X); dX = conjg(dX); }
          Ia[c] = Ia[c] + tm.coef * (X * s_);
          dIa[c] = dIa[c] + tm.coef * (dX * s_ + X * gs);
        }
      }
      cplx sl = mk(0, 0);
      for (int it = od.slp_ptr[lm]; it < od.slp_ptr[lm + 1]; ++it) {
        const Term tm = od.slp[it];
        cplx X = S.V[tm.n];
        if (tm.neg) X = conjg(X);
        sl = sl + tm.coef * (X * rget(S.Rt, tm.a, tm.b));
      }
      // gamma term: (-Omega_0, Omega_vec)(0, grad S^{lm}(x)), and its d/dnu'
      cplx g[3], hn[3];
      for (int a = 0; a < 3; ++a) {
        g[a] = dS(S.Rt, l, m, a);
        cplx acc = mk(0, 0);
        for (int b = 0; b < 3; ++b) acc = acc + S.nu[b] * d2S(S.Rt, l, m, a, b);
        hn[a] = acc;
      }
      const double o0 = -S.Om[0], o1 = S.Om[1], o2 = S.Om[2], o3 = S.Om[3];
      const double p0 = -S.dOm[0], p1 = S.dOm[1], p2 = S.dOm[2], p3 = S.dOm[3];
      // (s, w)(0, g) = (-w.g, s g + w x g)
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
        Dq[c] = -kSqrt2 * kInv4Pi * (Ia[c].im + Ig[c].im);
        dDq[c] = -kSqrt2 * kInv4Pi * (dIa[c].im + dIg[c].im);
      }
      const cplx Slm = S.Rt[tri(l, m)];
      const double Psi = kSqrt2 * kInv4Pi * (sl.im - Slm.im * S.Om[0]);
      // E = (0, nu') D = (-nu'.Dv, D0 nu' + nu' x Dv)
      const double n0_ = S.nu[0], n1_ = S.nu[1], n2_ = S.nu[2];
      double Eq[4];
      Eq[0] = -(n0_ * Dq[1] + n1_ * Dq[2] + n2_ * Dq[3]);
      Eq[1] = Dq[0] * n0_ + (n1_ * Dq[3] - n2_ * Dq[2]);
      Eq[2] = Dq[0] * n1_ + (n2_ * Dq[1] - n0_ * Dq[3]);
      Eq[3] = Dq[0] * n2_ + (n0_ * Dq[2] - n1_ * Dq[1]);
      const double sgn[4] = {1.0, -1.0, -1.0, -1.0};
      for (int c = 0; c < 4; ++c) {
        S.rD[c * NP + lm] = sgn[c] * Dq[c];
        S.rSp[c * NP + lm] = sgn[c] * Eq[c];
        S.rDp[c * NP + lm] = sgn[c] * dDq[c];
        S.rS[(c + 1) * NP + lm] = sgn[c] * Dq[c];
      }
      S.rS[lm] = Psi;
      // self target, principal value: D row -= 1/2 [(0, grad H(x)) .]_0,
      // S' row += 1/2 (-[(0,nu')(0, grad H(x)) .]_0)
      if (self >= 0 && (out.flags & RRQ_F_ONSURF_PV)) {
        const double gh0 = kSqrt2 * g[0].im, gh1 = kSqrt2 * g[1].im, gh2 = kSqrt2 * g[2].im;
        S.rD[1 * NP + lm] += 0.5 * gh0;
        S.rD[2 * NP + lm] += 0.5 * gh1;
        S.rD[3 * NP + lm] += 0.5 * gh2;
        S.rSp[0 * NP + lm] += 0.5 * (n0_ * gh0 + n1_ * gh1 + n2_ * gh2);
        S.rSp[1 * NP + lm] += 0.5 * (n1_ * gh2 - n2_ * gh1);
        S.rSp[2 * NP + lm] += 0.5 * (n2_ * gh0 - n0_ * gh2);
        S.rSp[3 * NP + lm] += 0.5 * (n0_ * gh1 - n1_ * gh0);
      }
    }
    __syncthreads();
    // weights = rows x maps (matrix-row remark after the algorithm), scale, correction
    const double* maps = pd.maps + pd.map_off[P];
    const double sc = S.fr[12];
    const int64_t ob = out.pair_off[k];
    const double x0 = tg.xyz[t], x1 = tg.xyz[tg.T + t], x2 = tg.xyz[2 * tg.T + t];
    const double nt0 = tg.nrm[t], nt1 = tg.nrm[tg.T + t], nt2 = tg.nrm[2 * tg.T + t];
    for (int idx = tid; idx < 4 * Q2; idx += PNT) {
      const int K = idx / Q2, j = idx % Q2;
      if (!(out.kmask & (1u << K)) || out.w[K] == nullptr) continue;
      double acc = 0.0;
      if (K == 0) {
        const double* M = maps + 8 * NP * Q2;
        for (int r = 0; r < 5 * NP; ++r) acc += S.rS[r] * M[r * Q2 + j];
        acc *= sc;
      } else if (K == 1) {
        for (int r = 0; r < 4 * NP; ++r) acc += S.rD[r] * maps[r * Q2 + j];
      } else if (K == 2) {
        const double* M = maps + 4 * NP * Q2;
        for (int r = 0; r < 4 * NP; ++r) acc += S.rSp[r] * M[r * Q2 + j];
      } else {
        for (int r = 0; r < 4 * NP; ++r) acc += S.rDp[r] * maps[r * Q2 + j];
        acc /= sc;
      }
      if ((out.flags & RRQ_F_CORRECTION) && j != self) {
        const int64_t nj = n0 + j;
        const double d0 = x0 - pd.node_xyz[nj], d1 = x1 - pd.node_xyz[pd.N + nj],
                     d2 = x2 - pd.node_xyz[2 * pd.N + nj];
        const double R2 = d0 * d0 + d1 * d1 + d2 * d2, R = sqrt(R2), R3 = R2 * R;
        const double v0 = pd.node_nrm[nj], v1 = pd.node_nrm[pd.N + nj], v2 = pd.node_nrm[2 * pd.N + nj];
        const double wj = pd.node_wt[nj] * kInv4Pi;
        const double dn = d0 * v0 + d1 * v1 + d2 * v2;
        const double dnt = d0 * nt0 + d1 * nt1 + d2 * nt2;
        double kv;
        if (K == 0) kv = 1.0 / R;
        else if (K == 1) kv = dn / R3;
        else if (K == 2) kv = -dnt / R3;
        else kv = (v0 * nt0 + v1 * nt1 + v2 * nt2) / R3 - 3.0 * dn * dnt / (R3 * R2);
        acc -= kv * wj;
      }
      if (!isfinite(acc)) {
        atomicAdd(&out.counters[kCNonfinite], 1ull);
        flag_pair(out.pflags, out.counters, k, kFlagNonfinite);
      }
      out.w[K][ob + j] = acc;
    }
  }
}

#define RRQ_FOR_ORDERS(X) X(4) X(5) X(6) X(8) X(10)

hipError_t launch_pair_plain(int q, const PlanDev& pd, const OrderDev& od, const TargetsDev& tg,
                             const AssembleOut& out, const SolveOpts& so, hipStream_t st) {
  if (tg.nnz <= 0) return hipSuccess;
  const int64_t g = tg.nnz < 1048576 ? tg.nnz : 1048576;
  switch (q) {
#define X(Q) case Q: hipLaunchKernelGGL(k_pair_plain<Q>, dim3((unsigned)g), dim3(PNT), 0, st, pd, od, tg, out, so); break;
    RRQ_FOR_ORDERS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// apply: pot[t] = sum over pairs of t of W[block] . density[nodes of P]
// ---------------------------------------------------------------------------------------
__global__ void k_apply(PlanDev pd, TargetsDev tg, const double* w0, const double* w1,
                        const double* w2, const double* w3, uint32_t kmask,
                        const int64_t* pair_off, const double* dens, double* p0, double* p1,
                        double* p2, double* p3) {
  const int64_t t = blockIdx.x;
  if (t >= tg.T) return;
  const double* W[4] = {w0, w1, w2, w3};
  double* Pp[4] = {p0, p1, p2, p3};
  __shared__ double red[4];
  for (int K = 0; K < 4; ++K) {
    if (!(kmask & (1u << K)) || W[K] == nullptr || Pp[K] == nullptr) continue;
    double acc = 0.0;
    // the row range and patch indices are clamped to the arrays' sizes (this call has no
    // validation word; rrq_pair_offsets checks the near list)
    const int64_t k0 = tg.near_ptr[t] > 0 ? tg.near_ptr[t] : 0;
    const int64_t k1 = tg.near_ptr[t + 1] < tg.nnz ? tg.near_ptr[t + 1] : tg.nnz;
    for (int64_t k = k0; k < k1; ++k) {
      const int P = tg.near_patch[k];
      if (P < 0 || P >= pd.npatch) continue;
      const int q2 = pd.order[P] * pd.order[P];
      const int64_t n0 = pd.node_off[P], ob = pair_off[k];
      for (int j = threadIdx.x; j < q2; j += blockDim.x) acc += W[K][ob + j] * dens[n0 + j];
    }
    const double s = block_sum<256>(acc, red);
    if (threadIdx.x == 0) Pp[K][t] = s;
  }
}

hipError_t launch_apply(const PlanDev& pd, const TargetsDev& tg, const double* const* w,
                        uint32_t kmask, const int64_t* pair_off, const int64_t*,
                        const double* density, double* const* pot, hipStream_t st) {
  if (tg.T <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_apply, dim3((unsigned)tg.T), dim3(256), 0, st, pd, tg, w[0], w[1], w[2],
                     w[3], kmask, pair_off, density, pot[0], pot[1], pot[2], pot[3]);
  return hipGetLastError();
}

}  // namespace rrq
