// Source-only kernels (Steps 1-3 of the algorithm in Sec. 4): patch frame and local
// coordinates, edge interpolants and edge tables, and the least-squares harmonic fits that
// give the nodal-to-coefficient maps of every patch.
#include "rrq_device.h"
#include "rrq_internal.h"

namespace rrq {

constexpr int NT = 256;

// ---------------------------------------------------------------------------------------
// Frame (Sec. 5.1 scaling/rotation): origin = mean of the corners, z along
// (c2 - c0) x (c3 - c1) (sign of the mean node normal), x along the first side, scale =
// longest side.  Local coordinates R^T (r - o) / s of nodes and edge samples; Legendre
// coefficients of each edge interpolant (discrete Legendre transform of the GL samples,
// a well-conditioned representation of the boundary curve) and its tangent.
// ---------------------------------------------------------------------------------------
template <int Q>
__global__ __launch_bounds__(NT) void k_geometry(PlanDev pd, rrq_surface s, OrderDev od,
                                                 const int32_t* patches, int count) {
  constexpr int PT = 2 * Q;
  __shared__ double sm_fr[kFrame];
  __shared__ double sm_c[4][3];
  __shared__ double sm_nrm[NT / 64 * 3];
  __shared__ double sm_loc[4 * PT * 3];
  __shared__ double sm_coef[4 * PT * 3];
  for (int it = blockIdx.x; it < count; it += gridDim.x) {
    const int P = patches[it];
    const int64_t n0 = s.node_off[P];
    const int64_t e0 = s.edge_off[P];
    const int tid = threadIdx.x;
    // corners c_e = r_e(-1) = sum_i l_i(-1) s_{e,i}
    if (tid < 12) {
      const int e = tid / 3, c = tid % 3;
      double acc = 0.0;
      for (int i = 0; i < PT; ++i) acc += od.lag_m1[i] * s.edge_xyz[c * s.nedge + e0 + e * PT + i];
      sm_c[e][c] = acc;
    }
    // mean node normal (only its direction's sign is used)
    double nx = 0, ny = 0, nz = 0;
    for (int i = tid; i < Q * Q; i += NT) {
      nx += s.node_nrm[0 * s.nnode + n0 + i];
      ny += s.node_nrm[1 * s.nnode + n0 + i];
      nz += s.node_nrm[2 * s.nnode + n0 + i];
    }
    nx = wave_sum(nx);
    ny = wave_sum(ny);
    nz = wave_sum(nz);
    if ((tid & 63) == 0) {
      sm_nrm[(tid >> 6) * 3 + 0] = nx;
      sm_nrm[(tid >> 6) * 3 + 1] = ny;
      sm_nrm[(tid >> 6) * 3 + 2] = nz;
    }
    __syncthreads();
    if (tid == 0) {
      double mn[3] = {0, 0, 0};
      for (int w = 0; w < NT / 64; ++w)
        for (int c = 0; c < 3; ++c) mn[c] += sm_nrm[w * 3 + c];
      double o[3], a[3], b[3], ez[3], ex[3], ey[3];
      for (int c = 0; c < 3; ++c) {
        o[c] = 0.25 * (sm_c[0][c] + sm_c[1][c] + sm_c[2][c] + sm_c[3][c]);
        a[c] = sm_c[2][c] - sm_c[0][c];
        b[c] = sm_c[3][c] - sm_c[1][c];
      }
      ez[0] = a[1] * b[2] - a[2] * b[1];
      ez[1] = a[2] * b[0] - a[0] * b[2];
      ez[2] = a[0] * b[1] - a[1] * b[0];
      double nn = sqrt(ez[0] * ez[0] + ez[1] * ez[1] + ez[2] * ez[2]);
      for (int c = 0; c < 3; ++c) ez[c] /= nn;
      if (ez[0] * mn[0] + ez[1] * mn[1] + ez[2] * mn[2] < 0)
        for (int c = 0; c < 3; ++c) ez[c] = -ez[c];
      double s1[3];
      for (int c = 0; c < 3; ++c) s1[c] = sm_c[1][c] - sm_c[0][c];
      double pz = s1[0] * ez[0] + s1[1] * ez[1] + s1[2] * ez[2];
      for (int c = 0; c < 3; ++c) ex[c] = s1[c] - pz * ez[c];
      nn = sqrt(ex[0] * ex[0] + ex[1] * ex[1] + ex[2] * ex[2]);
      for (int c = 0; c < 3; ++c) ex[c] /= nn;
      ey[0] = ez[1] * ex[2] - ez[2] * ex[1];
      ey[1] = ez[2] * ex[0] - ez[0] * ex[2];
      ey[2] = ez[0] * ex[1] - ez[1] * ex[0];
      double sc = 0.0;
      for (int e = 0; e < 4; ++e) {
        double d2 = 0;
        for (int c = 0; c < 3; ++c) {
          double d = sm_c[(e + 1) & 3][c] - sm_c[e][c];
          d2 += d * d;
        }
        sc = fmax(sc, sqrt(d2));
      }
      for (int c = 0; c < 3; ++c) {
        sm_fr[c] = o[c];
        sm_fr[3 + c] = ex[c];
        sm_fr[6 + c] = ey[c];
        sm_fr[9 + c] = ez[c];
      }
      sm_fr[12] = sc;
      for (int c = 13; c < kFrame; ++c) sm_fr[c] = 0.0;
    }
    __syncthreads();
    if (tid < kFrame) pd.frame[(int64_t)P * kFrame + tid] = sm_fr[tid];
    const double inv_s = 1.0 / sm_fr[12];
    for (int i = tid; i < Q * Q; i += NT) {
      double d[3], v[3];
      for (int c = 0; c < 3; ++c) {
        d[c] = s.node_xyz[c * s.nnode + n0 + i] - sm_fr[c];
        v[c] = s.node_nrm[c * s.nnode + n0 + i];
      }
      for (int a = 0; a < 3; ++a) {
        const double* ax = sm_fr + 3 + 3 * a;
        pd.node_loc[a * pd.N + n0 + i] = (d[0] * ax[0] + d[1] * ax[1] + d[2] * ax[2]) * inv_s;
        pd.node_loc[(3 + a) * pd.N + n0 + i] = v[0] * ax[0] + v[1] * ax[1] + v[2] * ax[2];
      }
    }
    for (int i = tid; i < 4 * PT; i += NT) {
      double d[3];
      for (int c = 0; c < 3; ++c) d[c] = s.edge_xyz[c * s.nedge + e0 + i] - sm_fr[c];
      for (int a = 0; a < 3; ++a) {
        const double* ax = sm_fr + 3 + 3 * a;
        double v = (d[0] * ax[0] + d[1] * ax[1] + d[2] * ax[2]) * inv_s;
        sm_loc[i * 3 + a] = v;
        pd.edge_loc[a * pd.E + e0 + i] = v;
      }
    }
    __syncthreads();
    // Legendre coefficients c_k = (2k+1)/2 sum_i w_i P_k(t_i) s_i per edge and coordinate
    for (int idx = tid; idx < 4 * PT * 3; idx += NT) {
      const int c = idx % 3, k = (idx / 3) % PT, e = idx / (3 * PT);
      double acc = 0.0;
      for (int i = 0; i < PT; ++i) acc += od.LT[k * PT + i] * sm_loc[(e * PT + i) * 3 + c];
      pd.edge_coef[c * pd.E + e0 + e * PT + k] = acc;
      sm_coef[(e * PT + k) * 3 + c] = acc;
    }
    __syncthreads();
    // chord of each edge (the start of the singularity-swap root search), by the same
    // arithmetic as from the global coefficients
    if (tid < 4) {
      double m[3], d[3];
      edge_chord(sm_coef + tid * PT * 3, PT, m, d, 3, 1);
      double* o = pd.edge_chord + ((int64_t)P * 4 + tid) * 6;
      for (int c = 0; c < 3; ++c) {
        o[c] = m[c];
        o[3 + c] = d[c];
      }
    }
    // tangent r'(t_i) = sum_k c_k P_k'(t_i)
    for (int idx = tid; idx < 4 * PT * 3; idx += NT) {
      const int c = idx % 3, i = (idx / 3) % PT, e = idx / (3 * PT);
      double der = 0.0;
      for (int k = 0; k < PT; ++k) der += od.DP[i * PT + k] * sm_coef[(e * PT + k) * 3 + c];
      pd.edge_tan[c * pd.E + e0 + e * PT + i] = der;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------
// Edge tables (Step 3): at every edge node r_i with tangent r'_i and every (j, k),
// 1 <= j <= p, 0 <= k <= j:  c = grad S^{jk}(r_i) x r'_i,  h = Hess S^{jk}(r_i) r'_i.
// ---------------------------------------------------------------------------------------
template <int Q>
__global__ __launch_bounds__(128) void k_edge_tables(PlanDev pd, OrderDev od,
                                                    const int32_t* patches, int count) {
  constexpr int PT = 2 * Q;
  constexpr int NJK = njk_of(Q);
  const int64_t total = (int64_t)count * 4 * PT;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int P = patches[g / (4 * PT)];
    const int ei = (int)(g % (4 * PT));
    const int e = ei / PT, i = ei % PT;
    const int64_t col = pd.edge_off[P] + ei;
    const double x = pd.edge_loc[0 * pd.E + col];
    const double y = pd.edge_loc[1 * pd.E + col];
    const double z = pd.edge_loc[2 * pd.E + col];
    const double tp[3] = {pd.edge_tan[0 * pd.E + col], pd.edge_tan[1 * pd.E + col],
                          pd.edge_tan[2 * pd.E + col]};
    cplx R[tri(Q, Q) + 1];
    solid_table<Q>(y, z, x, R);
    double* base = pd.tabs + pd.tab_off[P];
    for (int j = 1; j <= Q; ++j)
      for (int k = 0; k <= j; ++k) {
        cplx g3[3], h3[3];
        for (int a = 0; a < 3; ++a) {
          g3[a] = dS(R, j, k, a);
          cplx acc = mk(0, 0);
          for (int b = 0; b < 3; ++b) acc = acc + tp[b] * d2S(R, j, k, a, b);
          h3[a] = acc;
        }
        cplx c3[3];
        c3[0] = tp[2] * g3[1] - tp[1] * g3[2];
        c3[1] = tp[0] * g3[2] - tp[2] * g3[0];
        c3[2] = tp[1] * g3[0] - tp[0] * g3[1];
        // [edge node][component c0, c1, c2, h0, h1, h2][(j,k)] of (re, im) pairs: the (j,k)
        // of one node and component are contiguous
        double2* o = (double2*)base + ((int64_t)e * PT + i) * 6 * NJK + jk_index(j, k);
        for (int a = 0; a < 3; ++a) {
          o[a * NJK] = make_double2(c3[a].re, c3[a].im);
          o[(3 + a) * NJK] = make_double2(h3[a].re, h3[a].im);
        }
      }
  }
}

// ---------------------------------------------------------------------------------------
// Least squares by blocked Householder QR (compact WY form) on a row-major m x ncols matrix
// in global workspace: the first n columns are the system, the rest right-hand sides.
//  - each panel of HNB columns is copied to LDS and factorised by one wave (lane l owns the
//    panel rows r = l mod 64; reductions by lane exchanges, no workgroup barriers);
//  - its reflectors H_1 ... H_nb = I - V T V^T are applied to every later column in one pass
//    (C <- C - V T^T V^T C, one column per thread, loads issued 8 rows ahead);
//  - the right-hand sides are then solved with R by column sweeps, kBackCols columns at a
//    time held in LDS, with the columns of R staged in LDS kRC at a time.
// On exit the right-hand-side columns hold the solution in rows 0..n-1.
// LDS: V [m][HNB], T [HNB][HNB], G [HNB][HNB], beta [HNB], alpha [HNB], X [n][kBackCols],
// Rs [kRC][rs] (rs >= n).
// ---------------------------------------------------------------------------------------
constexpr int HNB = 8;
constexpr int kBackCols = 32;
constexpr int kRB = 8;   // rows per thread in the map products
constexpr int kRC = 8;   // columns of R staged in LDS per chunk of the back substitution

// Householder reflectors of one panel held in LDS (mr rows, nb <= HNB columns, row stride HNB),
// by wave 0: lane l owns the rows r = l mod 64; reductions by lane exchanges.  On exit the
// panel holds R above the diagonal and the reflectors below it; beta and alpha per column.
__device__ __forceinline__ void hh_panel(double* V, int mr, int nb, double* beta, double* alpha) {
  const int lane = threadIdx.x & 63;
    for (int c = 0; c < nb; ++c) {
      double part = 0.0;
      for (int r = lane; r < mr; r += 64)
        if (r >= c) {
          const double a = V[r * HNB + c];
          part += a * a;
        }
      const double nrm2 = wave_sum(part);
      const double akk = V[c * HNB + c];
      const double nrm = sqrt(nrm2);
      const double al = akk >= 0.0 ? -nrm : nrm;
      const double vtv = 2.0 * nrm * (nrm + fabs(akk));
      const double be = vtv > 0.0 ? 2.0 / vtv : 0.0;
      // w_j = v . V[:, j]; only c < j < nb are used (the others get 0: unchanged)
      double w[HNB];
#pragma unroll
      for (int j = 0; j < HNB; ++j) w[j] = 0.0;
      for (int r = lane; r < mr; r += 64)
        if (r >= c) {
          const double vr = r == c ? akk - al : V[r * HNB + c];
#pragma unroll
          for (int j = 0; j < HNB; ++j) w[j] += vr * V[r * HNB + j];
        }
#pragma unroll
      for (int j = 0; j < HNB; ++j) w[j] = (j > c && j < nb) ? be * wave_sum(w[j]) : 0.0;
      for (int r = lane; r < mr; r += 64)
        if (r >= c) {
          const double vr = r == c ? akk - al : V[r * HNB + c];
#pragma unroll
          for (int j = 0; j < HNB; ++j) V[r * HNB + j] -= w[j] * vr;
          if (r == c) V[r * HNB + c] = vr;
        }
      if (lane == 0) {
        beta[c] = be;
        alpha[c] = al;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

__device__ __forceinline__ void hh_lsq(double* A, int m, int n, int ncols, int ld, double* V0,
                                       double* V1, double* T, double* G, double* beta,
                                       double* alpha, double* X, double* Rs, int rs) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // the first panel; every later one is updated and factorised one step ahead (below)
  for (int idx = tid; idx < m * HNB; idx += NT) {
    const int r = idx / HNB, c = idx % HNB;
    V0[idx] = c < min(HNB, n) ? A[(int64_t)r * ld + c] : 0.0;
  }
  __syncthreads();
  if (wv == 0) hh_panel(V0, m, min(HNB, n), beta, alpha);
  __syncthreads();
  for (int k0 = 0, p = 0; k0 < n; k0 += HNB, ++p) {
    double* V = (p & 1) ? V1 : V0;    // this panel, factorised
    double* Vn = (p & 1) ? V0 : V1;   // the next one
    const int nb = min(HNB, n - k0);
    const int mr = m - k0;
    // R of the panel back to A (strict upper part from V, diagonal alpha); then V keeps only
    // the reflectors (zero above the diagonal)
    for (int idx = tid; idx < nb * nb; idx += NT) {
      const int r = idx / nb, c = idx % nb;
      if (r < c) A[(int64_t)(k0 + r) * ld + k0 + c] = V[r * HNB + c];
      else if (r == c) A[(int64_t)(k0 + r) * ld + k0 + c] = alpha[c];
    }
    __syncthreads();
    for (int idx = tid; idx < HNB * HNB; idx += NT) {
      const int r = idx / HNB, c = idx % HNB;
      if (r < c && r < mr) V[r * HNB + c] = 0.0;
    }
    __syncthreads();
    // G[l][i] = v_l . v_i for l < i, two threads per entry (alternate rows)
    {
      const int pidx = tid >> 1, h = tid & 1;
      int l = 0, i = 1, cnt = 0;
      for (int ii = 1; ii < HNB; ++ii)
        for (int ll = 0; ll < ii; ++ll, ++cnt)
          if (cnt == pidx) { l = ll; i = ii; }
      double g = 0.0;
      if (pidx < HNB * (HNB - 1) / 2 && i < nb)
        for (int r = i + h; r < mr; r += 2) g += V[r * HNB + l] * V[r * HNB + i];
      g += __shfl_xor(g, 1, 64);
      if (pidx < HNB * (HNB - 1) / 2 && h == 0) G[l * HNB + i] = g;
    }
    __syncthreads();
    // T (forward, columnwise): lane j of wave 0 builds row j of T in registers
    if (tid < HNB) {
      const int j = tid;
      double trow[HNB];
#pragma unroll
      for (int i = 0; i < HNB; ++i) {
        double v = 0.0;
        if (i < nb) {
          if (i == j) {
            v = beta[i];
          } else if (i > j) {
            double acc = 0.0;
#pragma unroll
            for (int l = 0; l < i; ++l)
              if (l >= j) acc += trow[l] * G[l * HNB + i];
            v = -beta[i] * acc;
          }
        }
        trow[i] = v;
      }
#pragma unroll
      for (int i = 0; i < HNB; ++i) T[j * HNB + i] = trow[i];
    }
    __syncthreads();
    // Look-ahead: wave 0 applies this panel's reflectors to the next panel's columns and
    // factorises that panel while waves 1-3 update the other later columns.  Every column is
    // updated with the same operations in the same order either way.
    const int k1 = k0 + nb;
    const bool ahead = k1 < n;
    if (ahead && wv == 0) {
      const int nb1 = min(HNB, n - k1);
      const int jj = lane >> 3, cc = lane & 7;   // next-panel column jj; reflector / row group cc
      const int j = k1 + jj;
      // w_cc of column j: one FMA chain over the rows in order
      double w = 0.0;
      if (jj < nb1) {
        int r = 0;
        for (; r + 8 <= mr; r += 8) {
          double a[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) a[u] = A[(int64_t)(k0 + r + u) * ld + j];
#pragma unroll
          for (int u = 0; u < 8; ++u) w = fma(V[(r + u) * HNB + cc], a[u], w);
        }
        for (; r < mr; ++r) w = fma(V[r * HNB + cc], A[(int64_t)(k0 + r) * ld + j], w);
      }
      double wl[HNB];
#pragma unroll
      for (int l = 0; l < HNB; ++l) wl[l] = __shfl(w, (lane & ~7) | l, 64);
      // T is upper triangular: the terms l > cc add exact zeros
      double acc = 0.0;
#pragma unroll
      for (int l = 0; l < HNB; ++l) acc = fma(T[l * HNB + cc], wl[l], acc);
      double wt[HNB];
#pragma unroll
      for (int c = 0; c < HNB; ++c) wt[c] = __shfl(acc, (lane & ~7) | c, 64);
      // rows r = cc mod 8 of column j: rows of this panel are R entries (back to A), the rest
      // become the next panel (zero columns past nb1)
      if (jj < nb1) {
        for (int r = cc; r < mr; r += 8) {
          double acc2 = 0.0;
#pragma unroll
          for (int c = 0; c < HNB; ++c) acc2 = fma(V[r * HNB + c], wt[c], acc2);
          const double v = A[(int64_t)(k0 + r) * ld + j] - acc2;
          if (r < nb) A[(int64_t)(k0 + r) * ld + j] = v;
          else Vn[(r - nb) * HNB + jj] = v;
        }
      } else {
        for (int r = nb + cc; r < mr; r += 8) Vn[(r - nb) * HNB + jj] = 0.0;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      hh_panel(Vn, mr - nb, nb1, beta, alpha);
    }
    // trailing update of the other later columns: C <- C - V T^T V^T C, one column per thread
    const int jbeg = ahead ? k1 + min(HNB, n - k1) : k1;
    const int tj = ahead ? tid - 64 : tid, tstep = ahead ? NT - 64 : NT;
    for (int j = jbeg + tj; tj >= 0 && j < ncols; j += tstep) {
      double w[HNB];
#pragma unroll
      for (int c = 0; c < HNB; ++c) w[c] = 0.0;
      int r = 0;
      for (; r + 8 <= mr; r += 8) {
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = A[(int64_t)(k0 + r + u) * ld + j];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          asm volatile("" ::: "memory");   // one row of V in registers at a time
#pragma unroll
          for (int c = 0; c < HNB; ++c) w[c] += V[(r + u) * HNB + c] * a[u];
        }
      }
      for (; r < mr; ++r) {
        const double a = A[(int64_t)(k0 + r) * ld + j];
#pragma unroll
        for (int c = 0; c < HNB; ++c) w[c] += V[r * HNB + c] * a;
      }
      double wt[HNB];
#pragma unroll
      for (int c = 0; c < HNB; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l <= c; ++l) acc += T[l * HNB + c] * w[l];
        wt[c] = acc;
      }
      r = 0;
      for (; r + 8 <= mr; r += 8) {
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = A[(int64_t)(k0 + r + u) * ld + j];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          asm volatile("" ::: "memory");
          double acc = 0.0;
#pragma unroll
          for (int c = 0; c < HNB; ++c) acc += V[(r + u) * HNB + c] * wt[c];
          A[(int64_t)(k0 + r + u) * ld + j] = a[u] - acc;
        }
      }
      for (; r < mr; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < HNB; ++c) acc += V[r * HNB + c] * wt[c];
        A[(int64_t)(k0 + r) * ld + j] -= acc;
      }
    }
    __syncthreads();
  }
  // back substitution R x = b for the right-hand sides, kBackCols columns per sweep
  for (int j0 = n; j0 < ncols; j0 += kBackCols) {
    const int cw = min(kBackCols, ncols - j0);
    for (int idx = tid; idx < n * kBackCols; idx += NT) {
      const int r = idx / kBackCols, jj = idx % kBackCols;
      X[idx] = jj < cw ? A[(int64_t)r * ld + j0 + jj] : 0.0;
    }
    // columns of R are staged in LDS kRC at a time (one barrier and one round of loads per
    // chunk); per column every thread divides its right-hand side's entry itself (the same
    // quotient in every thread of that column), updates its rows r < c, and after the
    // column's barrier one thread per right-hand side stores the quotient in row c
    const int jj = tid % kBackCols;
    double xc = 0.0;
    for (int cb = n; cb > 0; cb -= kRC) {
      const int clo = max(0, cb - kRC), nc = cb - clo;
      for (int idx = tid; idx < cb * nc; idx += NT) {
        const int r = idx / nc, cc = idx % nc;
        Rs[cc * rs + r] = A[(int64_t)r * ld + clo + cc];
      }
      __syncthreads();
      if (cb < n && tid < kBackCols) X[cb * kBackCols + tid] = xc;
      for (int c = cb - 1; c >= clo; --c) {
        const double* Rc = Rs + (c - clo) * rs;
        xc = X[c * kBackCols + jj] / Rc[c];
        for (int idx = tid; idx < c * kBackCols; idx += NT) X[idx] -= Rc[idx / kBackCols] * xc;
        __syncthreads();
        if (c > clo && tid < kBackCols) X[c * kBackCols + tid] = xc;
      }
    }
    if (tid < kBackCols) X[tid] = xc;
    __syncthreads();
    for (int idx = tid; idx < n * kBackCols; idx += NT) {
      const int r = idx / kBackCols, jj = idx % kBackCols;
      if (jj < cw) A[(int64_t)r * ld + j0 + jj] = X[idx];
    }
    __syncthreads();
  }
}

// sum of v over the workgroup (NT threads); every thread gets it.  red: NT / 64 doubles of LDS
__device__ __forceinline__ double fit_block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) t += red[i];
  __syncthreads();
  return t;
}

int64_t fit_ws_doubles(int q) {
  const int np = np_of(q), q2 = q * q;
  const int64_t a = (int64_t)(4 * q2) * (4 * np + q2);
  const int64_t b = (int64_t)q2 * (np + q2);
  return a + b + (int64_t)q2 * np + (int64_t)q2 * q2 + 64;
}

// ---------------------------------------------------------------------------------------
// Fits (Steps 1-2 with Step 2 skipped, remark after the algorithm):
//   DLP:  (0, grad H) c = (mu, 0) in the least-squares sense with weights w_a w_b
//         (block system of eq. dlpdensitylinearsystem2)  ->  M_D = A^+[:, block 0]
//   S':   right-hand side (0, sigma nu) (eq. sprimedensitylinearsystem): since the system
//         is quaternion-linear, column j of the map is (column j of M_D) * (0, nu_j)
//   SLP:  scalar system grad H . nu d = sigma (eq. slpdensitylinearsystem) -> B^+, and the
//         intermediate density rho = H d refitted by M_D (Theorem thm:slpreduction):
//         M_S = [B^+; M_D Hmat B^+]
// ---------------------------------------------------------------------------------------
template <int Q>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_fit(PlanDev pd, OrderDev od, const int32_t* patches,
                                            int count, double* ws, int64_t ws_per_block) {
  constexpr int NP = np_of(Q);
  constexpr int Q2 = Q * Q;
  constexpr int M = 4 * Q2;
  constexpr int LDA = 4 * NP + Q2;
  constexpr int LDB = NP + Q2;
  __shared__ double sV[2 * M * HNB];   // two panel buffers (look-ahead)
  __shared__ double sX[4 * NP * kBackCols];
  __shared__ double sR[kRC * 4 * NP];
  __shared__ double sT[HNB * HNB], sG[HNB * HNB], sbeta[HNB], salpha[HNB];
  __shared__ double sred[NT / 64];
  double* A = ws + (int64_t)blockIdx.x * ws_per_block;
  double* B = A + (int64_t)M * LDA;
  double* Hm = B + (int64_t)Q2 * LDB;
  double* T1 = Hm + (int64_t)Q2 * NP;
  for (int it = blockIdx.x; it < count; it += gridDim.x) {
    const int P = patches[it];
    const int64_t n0 = pd.node_off[P];
    const int tid = threadIdx.x;
    // clear workspace
    for (int64_t i = tid; i < (int64_t)M * LDA; i += NT) A[i] = 0.0;
    for (int64_t i = tid; i < (int64_t)Q2 * LDB; i += NT) B[i] = 0.0;
    __syncthreads();
    // basis at the nodes: one thread per node; squared Frobenius norms of the weighted
    // systems (the real DLP form holds each of F1, F2, F3 four times)
    double nA = 0.0, nB = 0.0;
    for (int i = tid; i < Q2; i += NT) {
      const double x = pd.node_loc[0 * pd.N + n0 + i];
      const double y = pd.node_loc[1 * pd.N + n0 + i];
      const double z = pd.node_loc[2 * pd.N + n0 + i];
      const double nu[3] = {pd.node_loc[3 * pd.N + n0 + i], pd.node_loc[4 * pd.N + n0 + i],
                            pd.node_loc[5 * pd.N + n0 + i]};
      const double om = sqrt(od.glq_w[i / Q] * od.glq_w[i % Q]);
      cplx R[tri(Q, Q) + 1];
      solid_table<Q>(y, z, x, R);
      int lm = 0;
      for (int l = 1; l <= Q; ++l)
        for (int m = 1; m <= l; ++m, ++lm) {
          double F[3];
          for (int a = 0; a < 3; ++a) F[a] = kSqrt2 * dS(R, l, m, a).im;
          Hm[i * NP + lm] = kSqrt2 * R[tri(l, m)].im;
          const double F1 = om * F[0], F2 = om * F[1], F3 = om * F[2];
          double* r0 = A + (int64_t)(0 * Q2 + i) * LDA;
          double* r1 = A + (int64_t)(1 * Q2 + i) * LDA;
          double* r2 = A + (int64_t)(2 * Q2 + i) * LDA;
          double* r3 = A + (int64_t)(3 * Q2 + i) * LDA;
          // [0 -F1 -F2 -F3; F1 0 -F3 F2; F2 F3 0 -F1; F3 -F2 F1 0]
          r0[1 * NP + lm] = -F1; r0[2 * NP + lm] = -F2; r0[3 * NP + lm] = -F3;
          r1[0 * NP + lm] = F1;  r1[2 * NP + lm] = -F3; r1[3 * NP + lm] = F2;
          r2[0 * NP + lm] = F2;  r2[1 * NP + lm] = F3;  r2[3 * NP + lm] = -F1;
          r3[0 * NP + lm] = F3;  r3[1 * NP + lm] = -F2; r3[2 * NP + lm] = F1;
          const double b = om * (F[0] * nu[0] + F[1] * nu[1] + F[2] * nu[2]);
          B[(int64_t)i * LDB + lm] = b;
          nA += 4.0 * (F1 * F1 + F2 * F2 + F3 * F3);
          nB += b * b;
        }
      A[(int64_t)i * LDA + 4 * NP + i] = om;
      B[(int64_t)i * LDB + NP + i] = om;
    }
    __syncthreads();
    hh_lsq(A, M, 4 * NP, LDA, LDA, sV, sV + M * HNB, sT, sG, sbeta, salpha, sX, sR, 4 * NP);
    hh_lsq(B, Q2, NP, LDB, LDB, sV, sV + M * HNB, sT, sG, sbeta, salpha, sX, sR, 4 * NP);
    // condition estimates: Frobenius-norm condition numbers ||A_w||_F ||A_w^+||_F, with
    // A_w^+ from the solutions (the maps over the weights; the three other block columns of
    // the DLP pseudoinverse are the same quaternions times i, j, k, hence the factor 4)
    double nAp = 0.0, nBp = 0.0;
    for (int idx = tid; idx < 4 * NP * Q2; idx += NT) {
      const int r = idx / Q2, j = idx % Q2;
      const double v = A[(int64_t)r * LDA + 4 * NP + j];
      nAp += 4.0 * v * v / (od.glq_w[j / Q] * od.glq_w[j % Q]);
    }
    for (int idx = tid; idx < NP * Q2; idx += NT) {
      const int r = idx / Q2, j = idx % Q2;
      const double v = B[(int64_t)r * LDB + NP + j];
      nBp += v * v / (od.glq_w[j / Q] * od.glq_w[j % Q]);
    }
    nA = fit_block_sum(nA, sred);
    nB = fit_block_sum(nB, sred);
    nAp = fit_block_sum(nAp, sred);
    nBp = fit_block_sum(nBp, sred);
    if (tid == 0) {
      pd.fitcond[2 * (int64_t)P] = sqrt(nA * nAp);
      pd.fitcond[2 * (int64_t)P + 1] = sqrt(nB * nBp);
    }
    double* maps = pd.maps + pd.map_off[P];
    double* MD = maps;
    double* MSp = maps + 4 * NP * Q2;
    double* MS = maps + 8 * NP * Q2;
    for (int idx = tid; idx < 4 * NP * Q2; idx += NT) {
      const int r = idx / Q2, j = idx % Q2;
      MD[idx] = A[(int64_t)r * LDA + 4 * NP + j];
    }
    for (int idx = tid; idx < NP * Q2; idx += NT) {
      const int r = idx / Q2, j = idx % Q2;
      MS[idx] = B[(int64_t)r * LDB + NP + j];
    }
    // T1 = Hmat (Q2 x NP) * B^+ (NP x Q2), kept in LDS (the panel or back-substitution
    // buffers, free now) where it fits.  Both products: one column j per lane and kRB rows per thread, so
    // that every loaded operand feeds kRB (or, for the row operand, one per row) FMAs; each
    // output is still one FMA chain in the order of the sum.
    constexpr bool kT1V = Q2 * Q2 <= 2 * M * HNB, kT1X = Q2 * Q2 <= 4 * NP * kBackCols;
    double* T1p = kT1V ? sV : (kT1X ? sX : T1);
    for (int it = tid; it < ((Q2 + kRB - 1) / kRB) * Q2; it += NT) {
      const int i0 = (it / Q2) * kRB, j = it % Q2;
      double acc[kRB];
#pragma unroll
      for (int u = 0; u < kRB; ++u) acc[u] = 0.0;
      for (int n = 0; n < NP; ++n) {
        const double b = B[(int64_t)n * LDB + NP + j];
#pragma unroll
        for (int u = 0; u < kRB; ++u)
          if (i0 + u < Q2) acc[u] = fma(Hm[(i0 + u) * NP + n], b, acc[u]);
      }
#pragma unroll
      for (int u = 0; u < kRB; ++u)
        if (i0 + u < Q2) T1p[(i0 + u) * Q2 + j] = acc[u];
    }
    __syncthreads();
    // M_S lower block = M_D * T1 ; M_Sp column j = (M_D column j) (0, nu_j)
    for (int it = tid; it < ((4 * NP + kRB - 1) / kRB) * Q2; it += NT) {
      const int r0 = (it / Q2) * kRB, j = it % Q2;
      double acc[kRB];
#pragma unroll
      for (int u = 0; u < kRB; ++u) acc[u] = 0.0;
      for (int i = 0; i < Q2; ++i) {
        const double t = T1p[i * Q2 + j];
#pragma unroll
        for (int u = 0; u < kRB; ++u)
          if (r0 + u < 4 * NP) acc[u] = fma(A[(int64_t)(r0 + u) * LDA + 4 * NP + i], t, acc[u]);
      }
#pragma unroll
      for (int u = 0; u < kRB; ++u)
        if (r0 + u < 4 * NP) MS[NP * Q2 + (r0 + u) * Q2 + j] = acc[u];
    }
    for (int idx = tid; idx < NP * Q2; idx += NT) {
      const int lm = idx / Q2, j = idx % Q2;
      const double c0 = A[(int64_t)(0 * NP + lm) * LDA + 4 * NP + j];
      const double c1 = A[(int64_t)(1 * NP + lm) * LDA + 4 * NP + j];
      const double c2 = A[(int64_t)(2 * NP + lm) * LDA + 4 * NP + j];
      const double c3 = A[(int64_t)(3 * NP + lm) * LDA + 4 * NP + j];
      const double v1 = pd.node_loc[3 * pd.N + n0 + j];
      const double v2 = pd.node_loc[4 * pd.N + n0 + j];
      const double v3 = pd.node_loc[5 * pd.N + n0 + j];
      MSp[(0 * NP + lm) * Q2 + j] = -(c1 * v1 + c2 * v2 + c3 * v3);
      MSp[(1 * NP + lm) * Q2 + j] = c0 * v1 + (c2 * v3 - c3 * v2);
      MSp[(2 * NP + lm) * Q2 + j] = c0 * v2 + (c3 * v1 - c1 * v3);
      MSp[(3 * NP + lm) * Q2 + j] = c0 * v3 + (c1 * v2 - c2 * v1);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------
// The DLP fit in quaternion arithmetic (orders whose system fits in LDS).  The real system
// of eq. dlpdensitylinearsystem2 is the real form of left multiplication by the pure
// quaternions F_{i,lm} = w_i (0, grad H^{lm}(r_i)) acting on c_lm = (c0, c1, c2, c3): block
// row r of A c is component r of sum_lm F_{i,lm} c_lm, and |.| of a quaternion is the
// 2-norm of its components, so the weighted least-squares problem is min ||F c - e|| over
// quaternion vectors c, with the right-hand sides e = w_j e_j (scalar quaternions).  It is
// solved by unpivoted Householder QR with quaternion reflectors H = I - beta v v^H (beta
// real), in LDS: a q^2 x n_p quaternion matrix holds 1/16 of the entries of the real form.
// Reflector of column k (entries x_i, i >= k): alpha = -u |x| with u = x_k / |x_k|,
// v = x - alpha e_k, beta = 1 / (|x| (|x| + |x_k|)); then v^H x = 1 / beta is real and
// H x = alpha e_k.  Column y: y - v (beta v^H y).  R_kk = alpha_k.
// ---------------------------------------------------------------------------------------
struct quat {
  double w, x, y, z;
};

__device__ __forceinline__ quat qmul(const quat& a, const quat& b) {
  return {a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z,
          a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
          a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x,
          a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}
// conj(a) b
__device__ __forceinline__ quat qcmul(const quat& a, const quat& b) {
  return {a.w * b.w + a.x * b.x + a.y * b.y + a.z * b.z,
          a.w * b.x - a.x * b.w - a.y * b.z + a.z * b.y,
          a.w * b.y + a.x * b.z - a.y * b.w - a.z * b.x,
          a.w * b.z - a.x * b.y + a.y * b.x - a.z * b.w};
}
__device__ __forceinline__ double qnorm2(const quat& a) {
  return a.w * a.w + a.x * a.x + a.y * a.y + a.z * a.z;
}

// beta v^H y of a reflector v (column of F from row k) and a column y, both at row stride ld
// (doubles): the eight lanes of a group (threadIdx.x mod 8) take rows k + g, k + g + 8, ...
// and their partial sums are added by three lane exchanges within the group
__device__ __forceinline__ quat reflect_coef(const double* v, int ldv, const double* y, int ldy,
                                            int k, int m, double beta) {
  quat a = {0.0, 0.0, 0.0, 0.0};
  for (int i = k + (threadIdx.x & 7); i < m; i += 8) {
    const quat t = qcmul(*(const quat*)(v + i * ldv), *(const quat*)(y + i * ldy));
    a.w += t.w; a.x += t.x; a.y += t.y; a.z += t.z;
  }
#pragma unroll
  for (int o = 1; o < 8; o <<= 1) {
    a.w += __shfl_xor(a.w, o, 64);
    a.x += __shfl_xor(a.x, o, 64);
    a.y += __shfl_xor(a.y, o, 64);
    a.z += __shfl_xor(a.z, o, 64);
  }
  return {beta * a.w, beta * a.x, beta * a.y, beta * a.z};
}

template <int Q>
struct FitQ {
  static constexpr int NP = np_of(Q), Q2 = Q * Q;
  // row strides (doubles) of the quaternion arrays: 16 bytes beyond whole quaternions, so
  // that the 16-byte reads of eight consecutive lanes (rows) of one column cover all 32 banks
  static constexpr int FS = 4 * NP + 2;
  static constexpr int o_F = 0;                          // [Q2][FS]: row i, column k at 4k
  static constexpr int o_Z = o_F + Q2 * FS;              // [Q2][FS]: Q_1, then the maps
  static constexpr int o_al = o_Z + Q2 * FS;             // [NP] quat: R_kk
  static constexpr int o_be = o_al + 4 * NP;             // [NP]
  static constexpr int n_quat = o_be + NP;
  // the SLP fit afterwards reuses the same LDS: panels, back-substitution right-hand
  // sides and R columns of hh_lsq for the Q2 x NP system, then T1 [Q2][Q2]
  static constexpr int o_sV = 0, o_sX = o_sV + 2 * Q2 * HNB, o_sR = o_sX + NP * kBackCols;
  static constexpr int o_sT = o_sR + kRC * NP, o_sG = o_sT + HNB * HNB,
                       o_sb = o_sG + HNB * HNB, o_sa = o_sb + HNB;
  static constexpr int n_slp = o_sa + HNB;
  static constexpr int n_t1 = Q2 * Q2;
  static constexpr int n_big = n_quat > n_slp ? (n_quat > n_t1 ? n_quat : n_t1)
                                              : (n_slp > n_t1 ? n_slp : n_t1);
  static constexpr int o_red = n_big;                    // [NT / 64] block sums
  static constexpr size_t bytes = (size_t)(n_big + NT / 64) * 8;
};

template <int Q>
__global__ __launch_bounds__(NT) void k_fit_quat(PlanDev pd, OrderDev od,
                                                 const int32_t* patches, int count, double* ws,
                                                 int64_t ws_per_block) {
  using L = FitQ<Q>;
  constexpr int NP = L::NP, Q2 = L::Q2;
  constexpr int LDB = NP + Q2;
  extern __shared__ double lds[];
  constexpr int FS = L::FS;
  auto Fq = [&](int i, int k) -> quat& { return *(quat*)(lds + L::o_F + i * FS + 4 * k); };
  auto Zq = [&](int i, int c) -> quat& { return *(quat*)(lds + L::o_Z + i * FS + 4 * c); };
  quat* al = (quat*)(lds + L::o_al);
  double* be = lds + L::o_be;
  // global workspace: the SLP system B [Q2][LDB] and Hmat [Q2][NP]
  double* B = ws + (int64_t)blockIdx.x * ws_per_block;
  double* Hm = B + (int64_t)Q2 * LDB;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int it = blockIdx.x; it < count; it += gridDim.x) {
    const int P = patches[it];
    const int64_t n0 = pd.node_off[P];
    __syncthreads();
    for (int64_t i = tid; i < (int64_t)Q2 * LDB; i += NT) B[i] = 0.0;
    __syncthreads();
    // basis at the nodes, one thread per node: F (LDS), B and Hmat (global); squared
    // Frobenius norms of the weighted systems
    double nF = 0.0, nB = 0.0;
    for (int i = tid; i < Q2; i += NT) {
      const double x = pd.node_loc[0 * pd.N + n0 + i];
      const double y = pd.node_loc[1 * pd.N + n0 + i];
      const double z = pd.node_loc[2 * pd.N + n0 + i];
      const double nu[3] = {pd.node_loc[3 * pd.N + n0 + i], pd.node_loc[4 * pd.N + n0 + i],
                            pd.node_loc[5 * pd.N + n0 + i]};
      const double om = sqrt(od.glq_w[i / Q] * od.glq_w[i % Q]);
      cplx R[tri(Q, Q) + 1];
      solid_table<Q>(y, z, x, R);
      int lm = 0;
      for (int l = 1; l <= Q; ++l)
        for (int m = 1; m <= l; ++m, ++lm) {
          double Fa[3];
          for (int a = 0; a < 3; ++a) Fa[a] = kSqrt2 * dS(R, l, m, a).im;
          Hm[i * NP + lm] = kSqrt2 * R[tri(l, m)].im;
          Fq(i, lm) = {0.0, om * Fa[0], om * Fa[1], om * Fa[2]};
          const double b = om * (Fa[0] * nu[0] + Fa[1] * nu[1] + Fa[2] * nu[2]);
          B[(int64_t)i * LDB + lm] = b;
          nF += om * om * (Fa[0] * Fa[0] + Fa[1] * Fa[1] + Fa[2] * Fa[2]);
          nB += b * b;
        }
      B[(int64_t)i * LDB + NP + i] = om;
    }
    double* red = lds + L::o_red;
    nF = fit_block_sum(nF, red);
    nB = fit_block_sum(nB, red);
    // quaternion Householder QR of F
    for (int k = 0; k < NP; ++k) {
      if (wv == 0) {
        double s2 = 0.0;
        for (int i = k + lane; i < Q2; i += 64) s2 += qnorm2(Fq(i, k));
        const double nrm = sqrt(wave_sum(s2));
        if (lane == 0) {
          const quat xk = Fq(k, k);
          const double ak = sqrt(qnorm2(xk));
          const quat u = ak > 0.0 ? quat{xk.w / ak, xk.x / ak, xk.y / ak, xk.z / ak}
                                  : quat{1.0, 0.0, 0.0, 0.0};
          if (nrm > 0.0) {
            al[k] = {-u.w * nrm, -u.x * nrm, -u.y * nrm, -u.z * nrm};
            be[k] = 1.0 / (nrm * (nrm + ak));
            const double f = ak + nrm;
            Fq(k, k) = {u.w * f, u.x * f, u.y * f, u.z * f};
          } else {
            al[k] = {0.0, 0.0, 0.0, 0.0};
            be[k] = 0.0;
          }
        }
      }
      __syncthreads();
      // later columns: threads = (column, group of rows i = k + g mod 8)
      const double bk = be[k];
      for (int j = k + 1 + (tid >> 3); j < NP; j += NT / 8) {
        const quat sv = reflect_coef(lds + L::o_F + 4 * k, FS, lds + L::o_F + 4 * j, FS, k, Q2,
                                     bk);
        for (int i = k + (tid & 7); i < Q2; i += 8) {
          const quat t = qmul(Fq(i, k), sv);
          quat& f = Fq(i, j);
          f.w -= t.w; f.x -= t.x; f.y -= t.y; f.z -= t.z;
        }
      }
      __syncthreads();
    }
    double nFp = 0.0;   // squared Frobenius norm of F^+ (maps over the weights), this thread's
    double* maps = pd.maps + pd.map_off[P];
    double* MD = maps;
    double* MSp = maps + 4 * NP * Q2;
    // F^+ = R^{-1} Q_1^H with Q_1 the first NP columns of Q = H_0 ... H_{NP-1}: Q_1 is
    // accumulated backwards (H_{NP-1} first) from [I; 0]; at step k the columns j < k are
    // still unit vectors with zeros in rows >= k, so only the columns j >= k change
    for (int idx = tid; idx < Q2 * NP; idx += NT) {
      const int i = idx / NP, j = idx % NP;
      Zq(i, j) = {i == j ? 1.0 : 0.0, 0.0, 0.0, 0.0};
    }
    __syncthreads();
    for (int k = NP - 1; k >= 0; --k) {
      const double bk = be[k];
      for (int j = k + (tid >> 3); j < NP; j += NT / 8) {
        const quat sv = reflect_coef(lds + L::o_F + 4 * k, FS, lds + L::o_Z + 4 * j, FS, k, Q2,
                                     bk);
        for (int i = k + (tid & 7); i < Q2; i += 8) {
          const quat t = qmul(Fq(i, k), sv);
          quat& z = Zq(i, j);
          z.w -= t.w; z.x -= t.x; z.y -= t.y; z.z -= t.z;
        }
      }
      __syncthreads();
    }
    // maps: column j of M_D is c = R^{-1} conj(Q_1[j, :])^T w_j, solved in place in row j of
    // Z for all j at once: c_k = R_kk^{-1} y_k, then y_l -= R_lk c_k for l < k
    for (int idx = tid; idx < Q2 * NP; idx += NT) {
      const int i = idx / NP, j = idx % NP;
      const double w = sqrt(od.glq_w[i / Q] * od.glq_w[i % Q]);
      quat& z = Zq(i, j);
      z = {w * z.w, -w * z.x, -w * z.y, -w * z.z};
    }
    __syncthreads();
    for (int k = NP - 1; k >= 0; --k) {
      if (tid < Q2) {
        const quat a = al[k];
        const double inv = 1.0 / qnorm2(a);
        const quat ai = {a.w * inv, -a.x * inv, -a.y * inv, -a.z * inv};
        Zq(tid, k) = qmul(ai, Zq(tid, k));
      }
      __syncthreads();
      for (int idx = tid; idx < k * Q2; idx += NT) {
        const int l = idx / Q2, j = idx % Q2;
        const quat t = qmul(Fq(l, k), Zq(j, k));
        quat& z = Zq(j, l);
        z.w -= t.w; z.x -= t.x; z.y -= t.y; z.z -= t.z;
      }
      __syncthreads();
    }
    // M_D columns (component-major rows b NP + lm) and M_Sp columns: c (0, nu_j)
    for (int idx = tid; idx < NP * Q2; idx += NT) {
      const int lm = idx / Q2, j = idx % Q2;
      const quat v = Zq(j, lm);
      nFp += qnorm2(v) / (od.glq_w[j / Q] * od.glq_w[j % Q]);
      MD[(0 * NP + lm) * Q2 + j] = v.w;
      MD[(1 * NP + lm) * Q2 + j] = v.x;
      MD[(2 * NP + lm) * Q2 + j] = v.y;
      MD[(3 * NP + lm) * Q2 + j] = v.z;
      const double v1 = pd.node_loc[3 * pd.N + n0 + j];
      const double v2 = pd.node_loc[4 * pd.N + n0 + j];
      const double v3 = pd.node_loc[5 * pd.N + n0 + j];
      MSp[(0 * NP + lm) * Q2 + j] = -(v.x * v1 + v.y * v2 + v.z * v3);
      MSp[(1 * NP + lm) * Q2 + j] = v.w * v1 + (v.y * v3 - v.z * v2);
      MSp[(2 * NP + lm) * Q2 + j] = v.w * v2 + (v.z * v1 - v.x * v3);
      MSp[(3 * NP + lm) * Q2 + j] = v.w * v3 + (v.x * v2 - v.y * v1);
    }
    __syncthreads();
    // SLP fit (real, Q2 x NP): blocked Householder in the same LDS
    hh_lsq(B, Q2, NP, LDB, LDB, lds + L::o_sV, lds + L::o_sV + Q2 * HNB, lds + L::o_sT,
           lds + L::o_sG, lds + L::o_sb, lds + L::o_sa, lds + L::o_sX, lds + L::o_sR, NP);
    double* MS = maps + 8 * NP * Q2;
    double nBp = 0.0;
    for (int idx = tid; idx < NP * Q2; idx += NT) {
      const int r = idx / Q2, j = idx % Q2;
      const double v = B[(int64_t)r * LDB + NP + j];
      MS[idx] = v;
      nBp += v * v / (od.glq_w[j / Q] * od.glq_w[j % Q]);
    }
    // condition estimates: Frobenius-norm condition numbers ||A_w||_F ||A_w^+||_F of the
    // weighted systems (the real DLP form has 4x the squared norms of the quaternion ones)
    nFp = fit_block_sum(nFp, red);
    nBp = fit_block_sum(nBp, red);
    if (tid == 0) {
      pd.fitcond[2 * (int64_t)P] = 4.0 * sqrt(nF * nFp);
      pd.fitcond[2 * (int64_t)P + 1] = sqrt(nB * nBp);
    }
    // T1 = Hmat (Q2 x NP) B^+ (NP x Q2) in LDS; M_S lower block = M_D T1 (M_D from the maps
    // just written: this workgroup's own stores)
    double* T1 = lds;
    for (int it2 = tid; it2 < ((Q2 + kRB - 1) / kRB) * Q2; it2 += NT) {
      const int i0 = (it2 / Q2) * kRB, j = it2 % Q2;
      double acc[kRB];
#pragma unroll
      for (int u = 0; u < kRB; ++u) acc[u] = 0.0;
      for (int n = 0; n < NP; ++n) {
        const double b = B[(int64_t)n * LDB + NP + j];
#pragma unroll
        for (int u = 0; u < kRB; ++u)
          if (i0 + u < Q2) acc[u] = fma(Hm[(i0 + u) * NP + n], b, acc[u]);
      }
#pragma unroll
      for (int u = 0; u < kRB; ++u)
        if (i0 + u < Q2) T1[(i0 + u) * Q2 + j] = acc[u];
    }
    __syncthreads();
    for (int it2 = tid; it2 < ((4 * NP + kRB - 1) / kRB) * Q2; it2 += NT) {
      const int r0 = (it2 / Q2) * kRB, j = it2 % Q2;
      double acc[kRB];
#pragma unroll
      for (int u = 0; u < kRB; ++u) acc[u] = 0.0;
      for (int i = 0; i < Q2; ++i) {
        const double t = T1[i * Q2 + j];
#pragma unroll
        for (int u = 0; u < kRB; ++u)
          if (r0 + u < 4 * NP) acc[u] = fma(MD[(r0 + u) * Q2 + i], t, acc[u]);
      }
#pragma unroll
      for (int u = 0; u < kRB; ++u)
        if (r0 + u < 4 * NP) MS[NP * Q2 + (r0 + u) * Q2 + j] = acc[u];
    }
    __syncthreads();
  }
}

#define RRQ_FOR_ORDERS(X) X(4) X(5) X(6) X(8) X(10)

hipError_t launch_geometry(const PlanDev& pd, const rrq_surface& s, const OrderDev& od,
                           const int32_t* patches, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int grid = count < 65535 ? count : 65535;
  switch (od.q) {
#define X(q) case q: hipLaunchKernelGGL(k_geometry<q>, dim3(grid), dim3(NT), 0, st, pd, s, od, patches, count); break;
    RRQ_FOR_ORDERS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_edge_tables(const PlanDev& pd, const OrderDev& od, const int32_t* patches,
                              int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int64_t total = (int64_t)count * 4 * od.pt;
  int64_t g = (total + 127) / 128;
  const int grid = (int)(g < 65535 ? g : 65535);
  switch (od.q) {
#define X(q) case q: hipLaunchKernelGGL(k_edge_tables<q>, dim3(grid), dim3(128), 0, st, pd, od, patches, count); break;
    RRQ_FOR_ORDERS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Orders whose quaternion DLP system fits in LDS take k_fit_quat; order 10 takes the real QR
// in global memory (k_fit).
template <int Q>
static hipError_t launch_fit_quat(const PlanDev& pd, const OrderDev& od, const int32_t* patches,
                                  int count, double* ws, int64_t ws_per_block, int grid,
                                  hipStream_t st) {
  const size_t lds = FitQ<Q>::bytes;
  static_assert(FitQ<Q>::bytes <= 160 * 1024, "quaternion fit exceeds the LDS");
  hipError_t e = hipFuncSetAttribute((const void*)k_fit_quat<Q>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  // at most one workgroup per compute unit: with more, the extra ones start only when a first
  // one has worked through all its patches, and the launch takes more rounds of patches
  if (lds > 80 * 1024) {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        ncu > 0 && grid > ncu)
      grid = ncu;
  }
  hipLaunchKernelGGL(k_fit_quat<Q>, dim3(grid), dim3(NT), lds, st, pd, od, patches, count, ws,
                     ws_per_block);
  return hipGetLastError();
}

hipError_t launch_fit(const PlanDev& pd, const OrderDev& od, const int32_t* patches, int count,
                      double* ws, int64_t ws_per_block, int blocks, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int grid = count < blocks ? count : blocks;
  switch (od.q) {
#define X(q) case q: return launch_fit_quat<q>(pd, od, patches, count, ws, ws_per_block, grid, st);
    X(4) X(5) X(6) X(8)
#undef X
    case 10:
      hipLaunchKernelGGL(k_fit<10>, dim3(grid), dim3(NT), 0, st, pd, od, patches, count, ws,
                         ws_per_block);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Non-finite entries in a patch's source-only data (frame, local nodes and normals, edge
// geometry, maps, edge tables): flags[P] = 1 if any, else 0.  One workgroup per patch.
__global__ void k_patch_check(PlanDev pd, int32_t* flags) {
  __shared__ int bad;
  for (int P = blockIdx.x; P < pd.npatch; P += gridDim.x) {
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    const int q = pd.order[P], q2 = q * q, pt = 2 * q;
    int b = 0;
    for (int i = threadIdx.x; i < 13; i += blockDim.x)   // o, ex, ey, ez, s
      b |= !isfinite(pd.frame[(int64_t)P * kFrame + i]);
    const int64_t n0 = pd.node_off[P], e0 = pd.edge_off[P];
    for (int i = threadIdx.x; i < 6 * q2; i += blockDim.x)
      b |= !isfinite(pd.node_loc[(int64_t)(i / q2) * pd.N + n0 + i % q2]);
    for (int i = threadIdx.x; i < 9 * 4 * pt; i += blockDim.x) {
      const int a = i / (12 * pt), r = i % (12 * pt);
      const double* arr = a == 0 ? pd.edge_loc : (a == 1 ? pd.edge_tan : pd.edge_coef);
      b |= !isfinite(arr[(int64_t)(r / (4 * pt)) * pd.E + e0 + r % (4 * pt)]);
    }
    const double* M = pd.maps + pd.map_off[P];
    for (int64_t i = threadIdx.x; i < map_doubles(q); i += blockDim.x) b |= !isfinite(M[i]);
    const double* tb = pd.tabs + pd.tab_off[P];
    for (int64_t i = threadIdx.x; i < tab_doubles(q); i += blockDim.x) b |= !isfinite(tb[i]);
    if (b) atomicOr(&bad, 1);
    __syncthreads();
    if (threadIdx.x == 0) flags[P] = bad;
    __syncthreads();
  }
}

hipError_t launch_patch_check(const PlanDev& pd, int32_t* flags, hipStream_t st) {
  const int grid = pd.npatch < 4096 ? pd.npatch : 4096;
  hipLaunchKernelGGL(k_patch_check, dim3(grid), dim3(256), 0, st, pd, flags);
  return hipGetLastError();
}

}  // namespace rrq
