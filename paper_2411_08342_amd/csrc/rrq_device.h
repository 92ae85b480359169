// Device helpers for the RRQ kernels: complex and quaternion arithmetic, regular solid
// harmonics (values by recurrence, derivatives by ladder identities), block reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace rrq {

constexpr double kPi = 3.14159265358979323846;
constexpr double kInv4Pi = 0.07957747154594766788;   // 1 / (4 pi)
constexpr double kSqrt2 = 1.41421356237309504880;

struct cplx {
  double re, im;
};

__device__ __forceinline__ cplx mk(double r, double i) { return cplx{r, i}; }
__device__ __forceinline__ cplx operator+(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx operator-(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx operator*(cplx a, cplx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cplx operator*(double s, cplx a) { return {s * a.re, s * a.im}; }
// 1/d from the hardware reciprocal estimate refined by one Newton step, r <- r + r (1 - d r)
// (for d finite and nonzero)
__device__ __forceinline__ double rcp_nr(double d) {
  const double r = __builtin_amdgcn_rcp(d);
  return fma(r, fma(-d, r, 1.0), r);
}
__device__ __forceinline__ cplx conjg(cplx a) { return {a.re, -a.im}; }
__device__ __forceinline__ double cabs2(cplx a) { return a.re * a.re + a.im * a.im; }
__device__ __forceinline__ double cabsd(cplx a) { return sqrt(a.re * a.re + a.im * a.im); }
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
  double s = 1.0 / (b.re * b.re + b.im * b.im);
  return {(a.re * b.re + a.im * b.im) * s, (a.im * b.re - a.re * b.im) * s};
}
// principal square root
__device__ __forceinline__ cplx csqrt(cplx z) {
  double r = sqrt(z.re * z.re + z.im * z.im);
  double a = sqrt(fmax(0.5 * (r + z.re), 0.0));
  double b = sqrt(fmax(0.5 * (r - z.re), 0.0));
  return {a, copysign(b, z.im)};
}

// Bernstein-ellipse radius of t w.r.t. [-1, 1] (the branch >= 1)
__device__ __forceinline__ double bernstein_rho(cplx t) {
  cplx s = csqrt(mk(t.re - 1.0, t.im)) * csqrt(mk(t.re + 1.0, t.im));
  double r = cabsd(t + s);
  if (!(r > 0.0)) return 1.0;
  return r >= 1.0 ? r : 1.0 / r;
}

// ---------------------------------------------------------------------------------------
// Regular solid harmonics R_l^m (Racah normalisation, no Condon-Shortley phase).
// Table holds m >= 0 at tri(l, m) = l(l+1)/2 + m.
// ---------------------------------------------------------------------------------------
__host__ __device__ constexpr int tri(int l, int m) { return l * (l + 1) / 2 + m; }

template <int L>
__device__ __forceinline__ void solid_table(double x, double y, double z, cplx* R) {
  const double r2 = x * x + y * y + z * z;
  R[0] = mk(1.0, 0.0);
#pragma unroll
  for (int l = 1; l <= L; ++l) {
    const double cd = sqrt((2.0 * l - 1.0) / (2.0 * l));
    cplx p = R[tri(l - 1, l - 1)];
    R[tri(l, l)] = mk(cd * (x * p.re - y * p.im), cd * (x * p.im + y * p.re));
#pragma unroll
    for (int m = 0; m < l; ++m) {
      const double inv = 1.0 / sqrt((double)(l * l - m * m));
      cplx a = R[tri(l - 1, m)];
      double c1 = (2.0 * l - 1.0) * z * inv;
      cplx v = c1 * a;
      if (m <= l - 2) {
        double c2 = r2 * sqrt((double)((l - 1 + m) * (l - 1 - m))) * inv;
        cplx b = R[tri(l - 2, m)];
        v = v - c2 * b;
      }
      R[tri(l, m)] = v;
    }
  }
}

// R_l^m for any m (R_l^{-m} = (-1)^m conj R_l^m); zero outside |m| <= l, l >= 0
__device__ __forceinline__ cplx rget(const cplx* R, int l, int m) {
  if (l < 0 || m > l || -m > l) return mk(0.0, 0.0);
  if (m >= 0) return R[tri(l, m)];
  cplx v = R[tri(l, -m)];
  return (m & 1) ? mk(-v.re, v.im) : mk(v.re, -v.im);
}

// ladder: op 0 = (dx + i dy), op 1 = (dx - i dy), op 2 = dz.  D_op R_l^m = c R_{l-1}^{m+dm}
__device__ __forceinline__ double ladder(int op, int l, int m, int* dm) {
  if (op == 0) {
    *dm = 1;
    if (m + 1 > l - 1 || -(m + 1) > l - 1) return 0.0;
    return -sqrt((double)((l - m) * (l - m - 1)));
  } else if (op == 1) {
    *dm = -1;
    if (m - 1 > l - 1 || -(m - 1) > l - 1) return 0.0;
    return sqrt((double)((l + m) * (l + m - 1)));
  }
  *dm = 0;
  if (m > l - 1 || -m > l - 1) return 0.0;
  return sqrt((double)((l + m) * (l - m)));
}

// Cartesian derivative d/dq_c of R_l^m at the tabulated point (c: 0 = x, 1 = y, 2 = z)
__device__ __forceinline__ cplx dR(const cplx* R, int l, int m, int c) {
  int dm;
  if (c == 2) {
    double k = ladder(2, l, m, &dm);
    return k == 0.0 ? mk(0, 0) : k * rget(R, l - 1, m);
  }
  int dp_, dn_;
  double kp = ladder(0, l, m, &dp_);
  double kn = ladder(1, l, m, &dn_);
  cplx P = kp == 0.0 ? mk(0, 0) : kp * rget(R, l - 1, m + 1);
  cplx N = kn == 0.0 ? mk(0, 0) : kn * rget(R, l - 1, m - 1);
  if (c == 0) return 0.5 * (P + N);
  cplx d = P - N;                       // -i/2 (P - N)
  return mk(0.5 * d.im, -0.5 * d.re);
}

// second derivative d^2/dq_c dq_e of R_l^m
__device__ __forceinline__ cplx d2R(const cplx* R, int l, int m, int c, int e) {
  // write d_c = sum_o T[c][o] D_o with T[x] = (1/2, 1/2, 0), T[y] = (-i/2, i/2, 0), T[z] = (0,0,1)
  cplx acc = mk(0, 0);
  for (int o1 = 0; o1 < 3; ++o1) {
    cplx t1;
    if (c == 0) t1 = o1 == 2 ? mk(0, 0) : mk(0.5, 0);
    else if (c == 1) t1 = o1 == 2 ? mk(0, 0) : (o1 == 0 ? mk(0, -0.5) : mk(0, 0.5));
    else t1 = o1 == 2 ? mk(1, 0) : mk(0, 0);
    if (t1.re == 0.0 && t1.im == 0.0) continue;
    for (int o2 = 0; o2 < 3; ++o2) {
      cplx t2;
      if (e == 0) t2 = o2 == 2 ? mk(0, 0) : mk(0.5, 0);
      else if (e == 1) t2 = o2 == 2 ? mk(0, 0) : (o2 == 0 ? mk(0, -0.5) : mk(0, 0.5));
      else t2 = o2 == 2 ? mk(1, 0) : mk(0, 0);
      if (t2.re == 0.0 && t2.im == 0.0) continue;
      int dm2, dm1;
      double k2 = ladder(o2, l, m, &dm2);
      if (k2 == 0.0) continue;
      double k1 = ladder(o1, l - 1, m + dm2, &dm1);
      if (k1 == 0.0) continue;
      acc = acc + (k1 * k2) * (t1 * t2 * rget(R, l - 2, m + dm2 + dm1));
    }
  }
  return acc;
}

// S^{lm}(x,y,z) = R_l^m(y,z,x).  The table must be built at q = (y, z, x).
// dS/dx_a = (dR/dq_{perm[a]})(q) with perm = (2, 0, 1).
__device__ __forceinline__ int sperm(int a) { return a == 0 ? 2 : a - 1; }
__device__ __forceinline__ cplx dS(const cplx* R, int l, int m, int a) {
  return dR(R, l, m, sperm(a));
}
__device__ __forceinline__ cplx d2S(const cplx* R, int l, int m, int a, int b) {
  return d2R(R, l, m, sperm(a), sperm(b));
}

// ---------------------------------------------------------------------------------------
// block reductions (blockDim = 256, wave64)
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  return s;
}

// value and derivative of the Legendre series sum_k coef[k*stride + c*cstride] P_k(t),
// c = 0..2, at complex t: P_{k+1} = ((2k+1) t P_k - k P_{k-1})/(k+1),
// P'_{k+1} = P'_{k-1} + (2k+1) P_k
__device__ __forceinline__ void leg3(const double* coef, int stride, int n, cplx t, cplx* r,
                                     cplx* dr, int64_t cstride = 1) {
  cplx p0 = mk(0, 0), p1 = mk(1, 0), d0 = mk(0, 0), d1 = mk(0, 0);
  for (int c = 0; c < 3; ++c) {
    r[c] = mk(coef[c * cstride], 0.0);
    dr[c] = mk(0, 0);
  }
  for (int k = 0; k < n - 1; ++k) {
    const cplx p2 = (1.0 / (k + 1)) * ((2.0 * k + 1.0) * (t * p1) - (double)k * p0);
    const cplx d2 = d0 + (2.0 * k + 1.0) * p1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    for (int c = 0; c < 3; ++c) {
      const double ck = coef[(k + 1) * stride + c * cstride];
      r[c] = r[c] + ck * p1;
      dr[c] = dr[c] + ck * d1;
    }
  }
}

// omega_0 integrand (eq. omega0def) per unit dt at a real parameter
__device__ __forceinline__ double omega0_at(const double* x, const double* u, const double* r,
                                            const double* dr) {
  const double d0 = x[0] - r[0], d1 = x[1] - r[1], d2 = x[2] - r[2];
  const double R = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  const double c0 = d1 * u[2] - d2 * u[1];
  const double c1 = d2 * u[0] - d0 * u[2];
  const double c2 = d0 * u[1] - d1 * u[0];
  const double num = c0 * dr[0] + c1 * dr[1] + c2 * dr[2];
  return num / (R * (R + d0 * u[0] + d1 * u[1] + d2 * u[2]));
}

// patch-local coordinates of a point: R^T (x - o) / s for the frame fr = o[3], e_x[3],
// e_y[3], e_z[3], s
__device__ __forceinline__ void frame_point(const double* fr, const double* x, double* xl) {
  const double inv_s = 1.0 / fr[12];
  const double dx[3] = {x[0] - fr[0], x[1] - fr[1], x[2] - fr[2]};
  for (int a = 0; a < 3; ++a) {
    const double* ax = fr + 3 + 3 * a;
    xl[a] = (dx[0] * ax[0] + dx[1] * ax[1] + dx[2] * ax[2]) * inv_s;
  }
}

// ---------------------------------------------------------------------------------------
// singularity-swap root (Sec. 3.5, Step 5): chord start and Newton on
// f(t) = sum_c (r_c(t) - x_c)^2 for an edge given by its Legendre coefficients
// cf[k ks + c cs] (ks = 3, cs = 1 for an interleaved copy; ks = 1, cs = E for the plan's
// component-major edge arrays)
// ---------------------------------------------------------------------------------------

// r(-1) and r(1) of the edge, then the chord midpoint m and half-vector d
__device__ __forceinline__ void edge_chord(const double* cf, int n, double* m, double* d,
                                           int ks = 3, int64_t cs = 1) {
  double A[3] = {0, 0, 0}, B[3] = {0, 0, 0};
  for (int kk = 0; kk < n; ++kk)
    for (int c = 0; c < 3; ++c) {
      const double v = cf[kk * ks + c * cs];
      A[c] += (kk & 1) ? -v : v;
      B[c] += v;
    }
  for (int c = 0; c < 3; ++c) {
    m[c] = 0.5 * (A[c] + B[c]);
    d[c] = 0.5 * (B[c] - A[c]);
  }
}

// root of the distance function of the straight chord
__device__ __forceinline__ cplx chord_root(const double* m, const double* d, const double* x) {
  const double v[3] = {x[0] - m[0], x[1] - m[1], x[2] - m[2]};
  const double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  const double cr0 = d[1] * v[2] - d[2] * v[1];
  const double cr1 = d[2] * v[0] - d[0] * v[2];
  const double cr2 = d[0] * v[1] - d[1] * v[0];
  return mk((d[0] * v[0] + d[1] * v[1] + d[2] * v[2]) / dd,
            sqrt(cr0 * cr0 + cr1 * cr1 + cr2 * cr2) / dd);
}

// Newton from t: returns 1 when the step fell below tol * max(1, |t|) within maxit
// iterations; *t is the last iterate (not canonicalised), *its the iterations taken
__device__ __forceinline__ int newton_solve(const double* cf, int n, const double* x, cplx* t,
                                            double tol, int maxit, int* its, int ks = 3,
                                            int64_t cs = 1) {
  cplx t0 = *t;
  int it;
  for (it = 1; it <= maxit; ++it) {
    cplx r[3], dr[3];
    leg3(cf, ks, n, t0, r, dr, cs);
    cplx f = mk(0, 0), fp = mk(0, 0);
    for (int c = 0; c < 3; ++c) {
      const cplx ec = r[c] - mk(x[c], 0.0);
      f = f + ec * ec;
      fp = fp + ec * dr[c];
    }
    const cplx dt = cdiv(f, 2.0 * fp);
    t0 = t0 - dt;
    if (cabsd(dt) <= tol * fmax(1.0, cabsd(t0))) {
      *t = t0;
      *its = it;
      return 1;
    }
  }
  *t = t0;
  *its = maxit;
  return 0;
}

// Features of (edge, target) for the learned initial guess: the chord root t_s, and the
// quadratic and cubic Legendre coefficients over |d| in the chord frame (e1 along d, e2
// toward the target's component perpendicular to the chord, e3 = e1 x e2).  Computed in
// double, returned rounded to float.
__device__ __forceinline__ void edge_features(const double* cf, int n, const double* x,
                                              float* f, cplx* ts_out, int ks = 3,
                                              int64_t cs = 1) {
  double m[3], d[3];
  edge_chord(cf, n, m, d, ks, cs);
  const cplx ts = chord_root(m, d, x);
  *ts_out = ts;
  const double ld = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  const double e1[3] = {d[0] / ld, d[1] / ld, d[2] / ld};
  const double v[3] = {x[0] - m[0], x[1] - m[1], x[2] - m[2]};
  const double ve = v[0] * e1[0] + v[1] * e1[1] + v[2] * e1[2];
  double e2[3] = {v[0] - ve * e1[0], v[1] - ve * e1[1], v[2] - ve * e1[2]};
  double nv = sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
  if (!(nv > 0.0)) {
    const double a[3] = {fabs(e1[0]) < 0.9 ? 1.0 : 0.0, fabs(e1[0]) < 0.9 ? 0.0 : 1.0, 0.0};
    const double ae = a[0] * e1[0] + a[1] * e1[1] + a[2] * e1[2];
    for (int c = 0; c < 3; ++c) e2[c] = a[c] - ae * e1[c];
    nv = sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
  }
  for (int c = 0; c < 3; ++c) e2[c] /= nv;
  const double e3[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                        e1[0] * e2[1] - e1[1] * e2[0]};
  f[0] = (float)ts.re;
  f[1] = (float)ts.im;
  for (int j = 0; j < 2; ++j) {
    double a[3] = {0, 0, 0};
    if (2 + j < n)
      for (int c = 0; c < 3; ++c) a[c] = cf[(2 + j) * ks + c * cs] / ld;
    f[2 + 3 * j] = (float)(a[0] * e1[0] + a[1] * e1[1] + a[2] * e1[2]);
    f[3 + 3 * j] = (float)(a[0] * e2[0] + a[1] * e2[1] + a[2] * e2[2]);
    f[4 + 3 * j] = (float)(a[0] * e3[0] + a[1] * e3[1] + a[2] * e3[2]);
  }
}

// Multilayer perceptron 8 -> 64 -> 64 -> 2 (tanh hidden units), float32 parameters, row-major
// [out][in] in this order: W1 [64][8], b1 [64], W2 [64][64], b2 [64], W3 [2][64], b3 [2]
constexpr int kMlpIn = 8, kMlpH = 64, kMlpOut = 2;
constexpr int kMlpParams = kMlpH * kMlpIn + kMlpH + kMlpH * kMlpH + kMlpH + kMlpOut * kMlpH + kMlpOut;
constexpr int kMlpW1 = 0, kMlpB1 = kMlpW1 + kMlpH * kMlpIn, kMlpW2 = kMlpB1 + kMlpH,
              kMlpB2 = kMlpW2 + kMlpH * kMlpH, kMlpW3 = kMlpB2 + kMlpH,
              kMlpB3 = kMlpW3 + kMlpOut * kMlpH;

}  // namespace rrq
