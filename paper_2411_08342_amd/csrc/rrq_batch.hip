// Batched form of the target-dependent steps: near pairs are binned by source patch on the
// device, and one workgroup assembles a tile of up to T targets of one patch, so that the
// patch's edge tables and coefficient maps are read once per tile and every phase has
// (target x something) parallelism.  Same arithmetic as the plain form, reorganised.
#include "rrq_device.h"
#include "rrq_internal.h"

namespace rrq {

constexpr int BNT = 256;
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kWavePanels = 64;

// ---------------------------------------------------------------------------------------
// binning: count pairs per patch, scan, scatter pair indices by patch, emit tiles
// ---------------------------------------------------------------------------------------
__global__ void k_bin_clear(int32_t* cnt, int32_t* fill, int P) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < P; i += gridDim.x * blockDim.x) {
    cnt[i] = 0;
    fill[i] = 0;
  }
}

__global__ void k_bin_count(TargetsDev tg, int32_t* cnt) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < tg.nnz;
       k += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&cnt[tg.near_patch[k]], 1);
}

// exclusive scans of cnt and of ceil(cnt / tile) over patches (one workgroup)
__global__ __launch_bounds__(1024) void k_bin_scan(const int32_t* cnt, int P, int tile,
                                                   int64_t* start, int64_t* tstart,
                                                   int64_t* ntiles) {
  __shared__ int64_t s1[1024], s2[1024];
  __shared__ int64_t c1, c2;
  if (threadIdx.x == 0) { c1 = 0; c2 = 0; }
  __syncthreads();
  for (int base = 0; base < P; base += 1024) {
    const int i = base + threadIdx.x;
    const int64_t a = i < P ? cnt[i] : 0;
    const int64_t b = i < P ? (cnt[i] + tile - 1) / tile : 0;
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int64_t x = threadIdx.x >= o ? s1[threadIdx.x - o] : 0;
      const int64_t y = threadIdx.x >= o ? s2[threadIdx.x - o] : 0;
      __syncthreads();
      s1[threadIdx.x] += x;
      s2[threadIdx.x] += y;
      __syncthreads();
    }
    if (i < P) {
      start[i] = c1 + s1[threadIdx.x] - a;
      tstart[i] = c2 + s2[threadIdx.x] - b;
    }
    __syncthreads();
    if (threadIdx.x == 1023) { c1 += s1[1023]; c2 += s2[1023]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    start[P] = c1;
    tstart[P] = c2;
    *ntiles = c2;
  }
}

__global__ void k_bin_scatter(TargetsDev tg, const int64_t* start, int32_t* fill,
                              int64_t* sorted) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < tg.nnz;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int P = tg.near_patch[k];
    const int pos = atomicAdd(&fill[P], 1);
    sorted[start[P] + pos] = k;
  }
}

__global__ void k_bin_tiles(const int32_t* cnt, int P, int tile, const int64_t* start,
                            const int64_t* tstart, int4* tiles) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
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

hipError_t launch_binning(const TargetsDev& tg, int P, int tile, int32_t* cnt, int32_t* fill,
                          int64_t* start, int64_t* tstart, int64_t* ntiles, int64_t* sorted,
                          int4* tiles, hipStream_t st) {
  const int gp = (P + 255) / 256;
  int64_t gk = (tg.nnz + 255) / 256;
  if (gk < 1) gk = 1;
  const unsigned gkk = (unsigned)(gk < 65535 ? gk : 65535);
  hipLaunchKernelGGL(k_bin_clear, dim3(gp), dim3(256), 0, st, cnt, fill, P);
  hipLaunchKernelGGL(k_bin_count, dim3(gkk), dim3(256), 0, st, tg, cnt);
  hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, st, cnt, P, tile, start, tstart, ntiles);
  hipLaunchKernelGGL(k_bin_scatter, dim3(gkk), dim3(256), 0, st, tg, start, fill, sorted);
  hipLaunchKernelGGL(k_bin_tiles, dim3(gp), dim3(256), 0, st, cnt, P, tile, start, tstart, tiles);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// LDS layout of one tile (doubles, then ints)
// ---------------------------------------------------------------------------------------
template <int Q, int T>
struct TileLds {
  static constexpr int PT = 2 * Q, NP = np_of(Q), NJK = njk_of(Q), NR = tri(Q, Q) + 1;
  static constexpr int o_fr = 0;
  static constexpr int o_eloc = o_fr + kFrame;
  static constexpr int o_etan = o_eloc + 4 * PT * 3;
  static constexpr int o_ecoef = o_etan + 4 * PT * 3;
  static constexpr int o_x = o_ecoef + 4 * PT * 3;        // [T][3]
  static constexpr int o_nu = o_x + 3 * T;
  static constexpr int o_u = o_nu + 3 * T;
  static constexpr int o_t0 = o_u + 3 * T;                 // [T][4][2]
  static constexpr int o_om = o_t0 + 8 * T;                // [T][4]: Omega_0, Omega_vec
  static constexpr int o_dom = o_om + 4 * T;               // [T][4]
  static constexpr int o_om0e = o_dom + 4 * T;             // [T][4]: Omega_0 of near edges
  static constexpr int o_td = o_om0e + 4 * T;              // [T][4][PT][8] (aliased by rows)
  static constexpr int n_td = T * 4 * PT * 8;
  static constexpr int o_lam = o_td + n_td;                // [T][4][PT][2]
  static constexpr int n_lam = T * 4 * PT * 2;
  static constexpr int n_rows = T * 17 * NP;
  static constexpr int n_scrA = (n_td + n_lam) > n_rows ? (n_td + n_lam) : n_rows;
  static constexpr int o_rows = o_td;                      // rD [T][4NP], rSp, rS [T][5NP], rDp
  static constexpr int o_vq = o_td + n_scrA;               // [T][NJK][18]
  static constexpr int o_rt = o_vq + T * NJK * 18;         // [T][NR] cplx
  static constexpr int o_gs = o_rt + 2 * T * NR;           // [T][NR] cplx
  static constexpr int o_pan = o_gs + 2 * T * NR;          // [4 waves][kWavePanels][2]
  static constexpr int o_red = o_pan + 4 * kWavePanels * 2;
  static constexpr int n_dbl = o_red + 8;
  // ints
  static constexpr int i_near = 0;                         // [T][4]
  static constexpr int i_self = i_near + 4 * T;
  static constexpr int i_npan = i_self + T;                // [4 waves]
  static constexpr int n_int = i_npan + 4;
  static constexpr size_t bytes = (size_t)n_dbl * 8 + (size_t)n_int * 4 + 64;
};

template <int Q, int T>
__global__ __launch_bounds__(BNT) void k_pair_tile(PlanDev pd, OrderDev od, TargetsDev tg,
                                                   AssembleOut out, SolveOpts so,
                                                   const int4* tiles, const int64_t* ntiles_p,
                                                   const int64_t* sorted) {
  using L = TileLds<Q, T>;
  constexpr int PT = L::PT, NP = L::NP, NJK = L::NJK, NR = L::NR, Q2 = Q * Q;
  extern __shared__ double smem[];
  double* fr = smem + L::o_fr;
  double* eloc = smem + L::o_eloc;
  double* etan = smem + L::o_etan;
  double* ecoef = smem + L::o_ecoef;
  double* sx = smem + L::o_x;
  double* snu = smem + L::o_nu;
  double* su = smem + L::o_u;
  double* st0 = smem + L::o_t0;
  double* som = smem + L::o_om;
  double* sdom = smem + L::o_dom;
  double* som0e = smem + L::o_om0e;
  double* td = smem + L::o_td;
  double* lam = smem + L::o_lam;
  double* rows = smem + L::o_rows;
  double* vq = smem + L::o_vq;
  cplx* Rt = (cplx*)(smem + L::o_rt);
  cplx* gS = (cplx*)(smem + L::o_gs);
  double* pan = smem + L::o_pan;
  int* ints = (int*)(smem + L::n_dbl);
  int* snear = ints + L::i_near;
  int* sself = ints + L::i_self;
  int* snpan = ints + L::i_npan;

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t ntiles = *ntiles_p;
  for (int64_t ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
    const int4 tile = tiles[ti];
    const int P = tile.x;
    if (pd.order[P] != Q) continue;
    const int64_t n0 = pd.node_off[P], e0 = pd.edge_off[P];
    for (int sub = 0; sub < tile.z; sub += T) {
      const int nt = min(T, tile.z - sub);
      __syncthreads();
      // ---- patch data
      if (tid < kFrame) fr[tid] = pd.frame[(int64_t)P * kFrame + tid];
      for (int i = tid; i < 4 * PT * 3; i += BNT) {
        const int c = i % 3, ei = i / 3;
        eloc[i] = pd.edge_loc[c * pd.E + e0 + ei];
        etan[i] = pd.edge_tan[c * pd.E + e0 + ei];
        ecoef[i] = pd.edge_coef[c * pd.E + e0 + ei];
      }
      __syncthreads();
      // ---- targets: local coordinates, u (nearest node, lowest index on ties)
      if (tid < nt) {
        const int t = tid;
        const int64_t k = sorted[tile.y + sub + t];
        const int64_t g = out.owner[k];
        const int self = (tg.self_patch[g] == P) ? tg.self_node[g] : -1;
        sself[t] = self;
        const double inv_s = 1.0 / fr[12];
        double dx[3], nv[3], xl[3], nl[3];
        for (int c = 0; c < 3; ++c) {
          dx[c] = tg.xyz[c * tg.T + g] - fr[c];
          nv[c] = tg.nrm[c * tg.T + g];
        }
        for (int a = 0; a < 3; ++a) {
          const double* ax = fr + 3 + 3 * a;
          xl[a] = (dx[0] * ax[0] + dx[1] * ax[1] + dx[2] * ax[2]) * inv_s;
          nl[a] = nv[0] * ax[0] + nv[1] * ax[1] + nv[2] * ax[2];
          sx[t * 3 + a] = xl[a];
          snu[t * 3 + a] = nl[a];
        }
        if (self >= 0) {
          for (int c = 0; c < 3; ++c) su[t * 3 + c] = nl[c];
        } else {
          double bd = 1e300;
          int bi = 0;
          for (int i = 0; i < Q2; ++i) {
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
          for (int c = 0; c < 3; ++c) su[t * 3 + c] = sg * nn[c];
        }
      }
      __syncthreads();
      // ---- Step 5: per (target, edge) classification and Newton root
      if (tid < 4 * nt) {
        const int t = tid >> 2, e = tid & 3;
        const double* cf = ecoef + e * PT * 3;
        const double* xl = sx + t * 3;
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
          v[c] = xl[c] - m[c];
        }
        const double dd = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
        const double cr0 = dv[1] * v[2] - dv[2] * v[1];
        const double cr1 = dv[2] * v[0] - dv[0] * v[2];
        const double cr2 = dv[0] * v[1] - dv[1] * v[0];
        const cplx ts = mk((dv[0] * v[0] + dv[1] * v[1] + dv[2] * v[2]) / dd,
                           sqrt(cr0 * cr0 + cr1 * cr1 + cr2 * cr2) / dd);
        int near = 0;
        cplx t0 = ts;
        if (bernstein_rho(ts) <= so.rho_far) {
          int conv = 0, its;
          for (its = 1; its <= so.newton_maxit; ++its) {
            cplx r[3], dr[3];
            leg3(cf, 3, PT, t0, r, dr);
            cplx f = mk(0, 0), fp = mk(0, 0);
            for (int c = 0; c < 3; ++c) {
              const cplx ec = r[c] - mk(xl[c], 0.0);
              f = f + ec * ec;
              fp = fp + ec * dr[c];
            }
            const cplx dt = cdiv(f, 2.0 * fp);
            t0 = t0 - dt;
            if (cabsd(dt) <= so.newton_tol * fmax(1.0, cabsd(t0))) { conv = 1; break; }
          }
          if (its > so.newton_maxit) its = so.newton_maxit;
          if (t0.im < 0) t0.im = -t0.im;
          if (conv && bernstein_rho(t0) <= so.rho_far) near = 1;
          atomicAdd(&out.counters[1], (unsigned long long)its);
          if (!conv) atomicAdd(&out.counters[2], 1ull);
          atomicMax(&out.counters[4], (unsigned long long)its);
          if (near) atomicAdd(&out.counters[0], 1ull);
        }
        snear[t * 4 + e] = near;
        st0[(t * 4 + e) * 2] = t0.re;
        st0[(t * 4 + e) * 2 + 1] = t0.im;
        som0e[t * 4 + e] = 0.0;
      }
      __syncthreads();
      // ---- Lagrange-basis moments of near edges on graded panels: one wave per near item
      for (int item = wv; item < 4 * nt; item += BNT / 64) {
        if (!snear[item]) continue;          // wave-uniform
        const int t = item >> 2, e = item & 3;
        const double a = st0[item * 2], b = st0[item * 2 + 1];
        double* wpan = pan + wv * kWavePanels * 2;
        if (lane == 0) {
          double stk[64][3];
          int sp = 0, np_ = 0;
          stk[0][0] = -1.0; stk[0][1] = 1.0; stk[0][2] = 0; sp = 1;
          while (sp > 0) {
            --sp;
            const double lo = stk[sp][0], hi = stk[sp][1];
            const int lev = (int)stk[sp][2];
            const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
            const double rho = bernstein_rho(mk((a - c) / h, b / h));
            if (lev >= 60 || rho >= so.rho_far || sp >= 62) {
              if (np_ < kWavePanels) { wpan[np_ * 2] = lo; wpan[np_ * 2 + 1] = hi; ++np_; }
              else atomicAdd(&out.counters[2], 1ull);
            } else {
              stk[sp][0] = c; stk[sp][1] = hi; stk[sp][2] = lev + 1; ++sp;
              stk[sp][0] = lo; stk[sp][1] = c; stk[sp][2] = lev + 1; ++sp;
            }
          }
          snpan[wv] = np_;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const int npts = snpan[wv] * PT;
        double l1acc = 0.0, l3acc = 0.0, om = 0.0;   // lane i < PT keeps lambda_i
        for (int base = 0; base < npts; base += 64) {
          const int idx = base + lane;
          double w1p = 0.0, w3p = 0.0, tau = 3.0;
          int hit = -2;
          if (idx < npts) {
            const int pn = idx / PT, g = idx % PT;
            const double lo = wpan[pn * 2], hi = wpan[pn * 2 + 1];
            const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
            tau = c + h * od.gl_t[g];
            const double K2 = (tau - a) * (tau - a) + b * b;
            const double K1 = 1.0 / sqrt(K2);
            const double hw = h * od.gl_w[g];
            double den = 0.0;
            hit = -1;
            for (int j = 0; j < PT; ++j) {
              const double dtj = tau - od.gl_t[j];
              if (dtj == 0.0) hit = j;
              else den += od.bary[j] / dtj;
            }
            w1p = hit >= 0 ? hw * K1 : hw * K1 / den;
            w3p = w1p / K2;
            cplx r[3], dr[3];
            leg3(ecoef + e * PT * 3, 3, PT, mk(tau, 0.0), r, dr);
            const double rr[3] = {r[0].re, r[1].re, r[2].re};
            const double ddd[3] = {dr[0].re, dr[1].re, dr[2].re};
            om += hw * omega0_at(sx + t * 3, su + t * 3, rr, ddd);
          }
          for (int i = 0; i < PT; ++i) {
            double li;
            if (hit >= 0) li = hit == i ? 1.0 : 0.0;
            else if (hit == -1) li = od.bary[i] / (tau - od.gl_t[i]);
            else li = 0.0;
            const double s1 = wave_sum(w1p * li);
            const double s3 = wave_sum(w3p * li);
            if (lane == i) { l1acc += s1; l3acc += s3; }
          }
        }
        om = wave_sum(om);
        if (lane < PT) {
          lam[((t * 4 + e) * PT + lane) * 2] = l1acc;
          lam[((t * 4 + e) * PT + lane) * 2 + 1] = l3acc;
        }
        if (lane == 0) som0e[item] = om;
        __builtin_amdgcn_wave_barrier();
      }
      __syncthreads();
      // ---- effective weights per (target, edge, node) and the Omega sums per (target, edge)
      if (tid < 4 * nt) {
        const int t = tid >> 2, e = tid & 3;
        const double* xl = sx + t * 3;
        const double* nl = snu + t * 3;
        const int near = snear[tid];
        const double a = st0[tid * 2], b = st0[tid * 2 + 1];
        double om0 = near ? som0e[tid] : 0.0;
        double ov[3] = {0, 0, 0}, dv[3] = {0, 0, 0}, dom0 = 0.0;
        for (int i = 0; i < PT; ++i) {
          const int ei = e * PT + i;
          double d[3];
          for (int c = 0; c < 3; ++c) d[c] = xl[c] - eloc[ei * 3 + c];
          const double R2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
          const double R = sqrt(R2);
          double w1, w3;
          if (near) {
            const double ta = od.gl_t[i] - a;
            const double q1 = sqrt(ta * ta + b * b) / R;
            w1 = lam[(tid * PT + i) * 2] * q1;
            w3 = lam[(tid * PT + i) * 2 + 1] * q1 * q1 * q1;
          } else {
            w1 = od.gl_w[i] / R;
            w3 = od.gl_w[i] / (R2 * R);
            om0 += od.gl_w[i] * omega0_at(xl, su + t * 3, eloc + ei * 3, etan + ei * 3);
          }
          const double dn = d[0] * nl[0] + d[1] * nl[1] + d[2] * nl[2];
          double* o = td + (tid * PT + i) * 8;
          o[0] = w1;
          for (int c = 0; c < 3; ++c) {
            o[1 + c] = d[c];
            o[4 + c] = w1 * nl[c] - w3 * dn * d[c];
          }
          const double* rp = etan + ei * 3;
          for (int c = 0; c < 3; ++c) {
            ov[c] -= w1 * rp[c];
            dv[c] += w3 * dn * rp[c];
          }
          const double cx = rp[1] * d[2] - rp[2] * d[1];
          const double cy = rp[2] * d[0] - rp[0] * d[2];
          const double cz = rp[0] * d[1] - rp[1] * d[0];
          dom0 -= w3 * (cx * nl[0] + cy * nl[1] + cz * nl[2]);
        }
        // per-(t,e) partials into lambda slots (dead now): reuse som0e for Omega_0
        som0e[tid] = om0;
        double* pp = lam + tid * PT * 2;   // PT*2 >= 7
        pp[0] = ov[0]; pp[1] = ov[1]; pp[2] = ov[2];
        pp[3] = dv[0]; pp[4] = dv[1]; pp[5] = dv[2]; pp[6] = dom0;
      }
      __syncthreads();
      if (tid < nt) {
        const int t = tid;
        double o[4] = {0, 0, 0, 0}, d[4] = {0, 0, 0, 0};
        for (int e = 0; e < 4; ++e) {
          const double* pp = lam + (t * 4 + e) * PT * 2;
          o[0] += som0e[t * 4 + e];
          o[1] += pp[0]; o[2] += pp[1]; o[3] += pp[2];
          d[1] += pp[3]; d[2] += pp[4]; d[3] += pp[5]; d[0] += pp[6];
        }
        for (int c = 0; c < 4; ++c) { som[t * 4 + c] = o[c]; sdom[t * 4 + c] = d[c]; }
      }
      // ---- Step 6: contraction with the edge tables, items (j,k) x target
      const double* tb = pd.tabs + pd.tab_off[P];
      for (int idx = tid; idx < NJK * T; idx += BNT) {
        const int n = idx / T, t = idx % T;
        if (t >= nt) continue;
        double V0 = 0, V1 = 0;
        double Qr[4] = {0, 0, 0, 0}, Qi[4] = {0, 0, 0, 0};
        double Dr[4] = {0, 0, 0, 0}, Di[4] = {0, 0, 0, 0};
        for (int e = 0; e < 4; ++e)
#pragma unroll 4
          for (int i = 0; i < PT; ++i) {
            const double* o = tb + (((int64_t)e * PT + i) * NJK + n) * 12;
            const double* tdp = td + ((t * 4 + e) * PT + i) * 8;
            const double w1 = tdp[0];
            const double d0 = tdp[1], d1 = tdp[2], d2 = tdp[3];
            const double a0 = tdp[4], a1 = tdp[5], a2 = tdp[6];
            const double c0r = o[0], c0i = o[1], c1r = o[2], c1i = o[3], c2r = o[4], c2i = o[5];
            const double h0r = o[6], h0i = o[7], h1r = o[8], h1i = o[9], h2r = o[10], h2i = o[11];
            V0 += w1 * (d0 * c0r + d1 * c1r + d2 * c2r);
            V1 += w1 * (d0 * c0i + d1 * c1i + d2 * c2i);
            const double v0 = w1 * d0, v1 = w1 * d1, v2 = w1 * d2;
            Qr[0] -= v0 * h0r + v1 * h1r + v2 * h2r;
            Qi[0] -= v0 * h0i + v1 * h1i + v2 * h2i;
            Qr[1] += v1 * h2r - v2 * h1r;
            Qi[1] += v1 * h2i - v2 * h1i;
            Qr[2] += v2 * h0r - v0 * h2r;
            Qi[2] += v2 * h0i - v0 * h2i;
            Qr[3] += v0 * h1r - v1 * h0r;
            Qi[3] += v0 * h1i - v1 * h0i;
            Dr[0] -= a0 * h0r + a1 * h1r + a2 * h2r;
            Di[0] -= a0 * h0i + a1 * h1i + a2 * h2i;
            Dr[1] += a1 * h2r - a2 * h1r;
            Di[1] += a1 * h2i - a2 * h1i;
            Dr[2] += a2 * h0r - a0 * h2r;
            Di[2] += a2 * h0i - a0 * h2i;
            Dr[3] += a0 * h1r - a1 * h0r;
            Di[3] += a0 * h1i - a1 * h0i;
          }
        double* o = vq + (t * NJK + n) * 18;
        o[0] = V0; o[1] = V1;
        for (int c = 0; c < 4; ++c) {
          o[2 + 2 * c] = Qr[c]; o[3 + 2 * c] = Qi[c];
          o[10 + 2 * c] = Dr[c]; o[11 + 2 * c] = Di[c];
        }
      }
      // ---- Step 4: target harmonics
      if (tid >= BNT - nt) {
        const int t = BNT - 1 - tid;
        solid_table<Q>(sx[t * 3 + 1], sx[t * 3 + 2], sx[t * 3 + 0], Rt + t * NR);
      }
      __syncthreads();
      for (int idx = tid; idx < nt * NR; idx += BNT) {
        const int t = idx / NR, r = idx % NR;
        int a = 0;
        while (tri(a + 1, 0) <= r) ++a;
        const int b = r - tri(a, 0);
        cplx acc = mk(0, 0);
        for (int c = 0; c < 3; ++c) acc = acc + snu[t * 3 + c] * dS(Rt + t * NR, a, b, c);
        gS[idx] = acc;
      }
      __syncthreads();
      // ---- Steps 7-8: translation and rows, items (target, l, m)
      for (int idx = tid; idx < nt * NP; idx += BNT) {
        const int t = idx / NP, lm = idx % NP;
        int l = 1;
        while (np_of(l) <= lm) ++l;
        const int m = lm - np_of(l - 1) + 1;
        const cplx* R = Rt + t * NR;
        const cplx* G = gS + t * NR;
        const double* VQ = vq + t * NJK * 18;
        cplx Ia[4] = {mk(0, 0), mk(0, 0), mk(0, 0), mk(0, 0)};
        cplx dIa[4] = {mk(0, 0), mk(0, 0), mk(0, 0), mk(0, 0)};
        for (int it = od.dlp_ptr[lm]; it < od.dlp_ptr[lm + 1]; ++it) {
          const Term tm = od.dlp[it];
          const cplx s_ = rget(R, tm.a, tm.b);
          cplx gs;
          if (tm.b >= 0) gs = G[tri(tm.a, tm.b)];
          else {
            const cplx g = G[tri(tm.a, -tm.b)];
            gs = ((-tm.b) & 1) ? mk(-g.re, g.im) : mk(g.re, -g.im);
          }
          const double* q = VQ + tm.n * 18;
          for (int c = 0; c < 4; ++c) {
            cplx X = mk(q[2 + 2 * c], q[3 + 2 * c]), dX = mk(q[10 + 2 * c], q[11 + 2 * c]);
            if (tm.neg) { X = conjg(X); dX = conjg(dX); }
            Ia[c] = Ia[c] + tm.coef * (X * s_);
            dIa[c] = dIa[c] + tm.coef * (dX * s_ + X * gs);
          }
        }
        cplx sl = mk(0, 0);
        for (int it = od.slp_ptr[lm]; it < od.slp_ptr[lm + 1]; ++it) {
          const Term tm = od.slp[it];
          const double* q = VQ + tm.n * 18;
          cplx X = mk(q[0], q[1]);
          if (tm.neg) X = conjg(X);
          sl = sl + tm.coef * (X * rget(R, tm.a, tm.b));
        }
        const double* nu = snu + t * 3;
        cplx g[3], hn[3];
        for (int a = 0; a < 3; ++a) {
          g[a] = dS(R, l, m, a);
          cplx acc = mk(0, 0);
          for (int b = 0; b < 3; ++b) acc = acc + nu[b] * d2S(R, l, m, a, b);
          hn[a] = acc;
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
          Dq[c] = -kSqrt2 * kInv4Pi * (Ia[c].im + Ig[c].im);
          dDq[c] = -kSqrt2 * kInv4Pi * (dIa[c].im + dIg[c].im);
        }
        const double Psi = kSqrt2 * kInv4Pi * (sl.im - R[tri(l, m)].im * som[t * 4]);
        const double n0_ = nu[0], n1_ = nu[1], n2_ = nu[2];
        double Eq[4];
        Eq[0] = -(n0_ * Dq[1] + n1_ * Dq[2] + n2_ * Dq[3]);
        Eq[1] = Dq[0] * n0_ + (n1_ * Dq[3] - n2_ * Dq[2]);
        Eq[2] = Dq[0] * n1_ + (n2_ * Dq[1] - n0_ * Dq[3]);
        Eq[3] = Dq[0] * n2_ + (n0_ * Dq[2] - n1_ * Dq[1]);
        double* rD = rows + t * 4 * NP;
        double* rSp = rows + T * 4 * NP + t * 4 * NP;
        double* rS = rows + T * 8 * NP + t * 5 * NP;
        double* rDp = rows + T * 13 * NP + t * 4 * NP;
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
      // ---- Step 8 (matrix rows): weights = rows x maps on FP64 MFMA 16x16x4.
      // Jobs (group, 16-column tile): group 0 = [rD; rDp] x M_D, 1 = rSp x M_Sp, 2 = rS x M_S.
      // MFMA operand layout: lane l holds A[l%16][l/16], B[l/16][l%16]; result element v of
      // lane l is D[l/16 + 4v][l%16].
      {
        constexpr int NCT = (Q2 + 15) / 16;
        const double* maps = pd.maps + pd.map_off[P];
        const double sc = fr[12];
        const int arow = lane & 15, akk = lane >> 4;
        for (int job = wv; job < 3 * NCT; job += BNT / 64) {
          const int grp = job / NCT, ct = job % NCT;
          const double* M = grp == 0 ? maps : (grp == 1 ? maps + 4 * NP * Q2 : maps + 8 * NP * Q2);
          const int KR = grp == 2 ? 5 * NP : 4 * NP;
          const double* rowp = nullptr;
          if (grp == 0) {
            if (arow < T) rowp = rows + arow * 4 * NP;
            else if (arow < 2 * T) rowp = rows + T * 13 * NP + (arow - T) * 4 * NP;
          } else if (arow < T) {
            rowp = grp == 1 ? rows + T * 4 * NP + arow * 4 * NP : rows + T * 8 * NP + arow * 5 * NP;
          }
          const int bcol = ct * 16 + (lane & 15);
          const bool bval = bcol < Q2;
          v4d acc = {0.0, 0.0, 0.0, 0.0};
          // 8 k-steps per batch: operands loaded first (8 map loads in flight), then 8 MFMAs
          for (int kb = 0; kb < KR; kb += 32) {
            double av[8], bv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int k = kb + 4 * u + akk;
              const bool ok = k < KR;
              av[u] = (rowp != nullptr && ok) ? rowp[k] : 0.0;
              bv[u] = (bval && ok) ? M[k * Q2 + bcol] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
              acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
          }
          if (!bval) continue;
          const int j = bcol;
          const int64_t nj = n0 + j;
          const double rx = pd.node_xyz[nj], ry = pd.node_xyz[pd.N + nj], rz = pd.node_xyz[2 * pd.N + nj];
          const double v0 = pd.node_nrm[nj], v1 = pd.node_nrm[pd.N + nj], v2 = pd.node_nrm[2 * pd.N + nj];
          const double wj = pd.node_wt[nj] * kInv4Pi;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = (lane >> 4) + 4 * v;
            int K, t;
            if (grp == 0) { K = i < T ? 1 : 3; t = i < T ? i : i - T; if (i >= 2 * T) t = T; }
            else { K = grp == 1 ? 2 : 0; t = i < T ? i : T; }
            if (t >= nt || !(out.kmask & (1u << K)) || out.w[K] == nullptr) continue;
            const int64_t k = sorted[tile.y + sub + t];
            const int64_t g = out.owner[k];
            double val = acc[v];
            if (K == 0) val *= sc;
            else if (K == 3) val /= sc;
            if ((out.flags & RRQ_F_CORRECTION) && j != sself[t]) {
              const double d0 = tg.xyz[g] - rx, d1 = tg.xyz[tg.T + g] - ry, d2 = tg.xyz[2 * tg.T + g] - rz;
              const double R2 = d0 * d0 + d1 * d1 + d2 * d2, R = sqrt(R2), R3 = R2 * R;
              const double nt0 = tg.nrm[g], nt1 = tg.nrm[tg.T + g], nt2 = tg.nrm[2 * tg.T + g];
              const double dn = d0 * v0 + d1 * v1 + d2 * v2;
              const double dnt = d0 * nt0 + d1 * nt1 + d2 * nt2;
              double kv;
              if (K == 0) kv = 1.0 / R;
              else if (K == 1) kv = dn / R3;
              else if (K == 2) kv = -dnt / R3;
              else kv = (v0 * nt0 + v1 * nt1 + v2 * nt2) / R3 - 3.0 * dn * dnt / (R3 * R2);
              val -= kv * wj;
            }
            out.w[K][out.pair_off[k] + j] = val;
          }
        }
      }
    }
  }
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

hipError_t launch_pair_tile(int q, int T, int grid, const PlanDev& pd, const OrderDev& od,
                            const TargetsDev& tg, const AssembleOut& out, const SolveOpts& so,
                            const int4* tiles, const int64_t* ntiles, const int64_t* sorted,
                            hipStream_t st) {
  if (tg.nnz <= 0) return hipSuccess;
  switch (q * 100 + T) {
#define X(Q, TT)                                                                               \
  case Q * 100 + TT: {                                                                        \
    const size_t lds = TileLds<Q, TT>::bytes;                                                 \
    static bool attr = false;                                                                 \
    if (!attr) {                                                                              \
      hipError_t e = hipFuncSetAttribute((const void*)k_pair_tile<Q, TT>,                     \
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
      if (e != hipSuccess) return e;                                                          \
      attr = true;                                                                            \
    }                                                                                         \
    hipLaunchKernelGGL((k_pair_tile<Q, TT>), dim3(grid), dim3(BNT), lds, st, pd, od, tg, out, \
                       so, tiles, ntiles, sorted);                                            \
    break;                                                                                    \
  }
    RRQ_TILE_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace rrq
