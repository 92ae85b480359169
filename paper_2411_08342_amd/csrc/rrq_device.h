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

// value and derivative of the Legendre series sum_k coef[k*stride + c] P_k(t), c = 0..2,
// at complex t: P_{k+1} = ((2k+1) t P_k - k P_{k-1})/(k+1), P'_{k+1} = P'_{k-1} + (2k+1) P_k
__device__ __forceinline__ void leg3(const double* coef, int stride, int n, cplx t, cplx* r,
                                     cplx* dr) {
  cplx p0 = mk(0, 0), p1 = mk(1, 0), d0 = mk(0, 0), d1 = mk(0, 0);
  for (int c = 0; c < 3; ++c) {
    r[c] = mk(coef[c], 0.0);
    dr[c] = mk(0, 0);
  }
  for (int k = 0; k < n - 1; ++k) {
    const cplx p2 = (1.0 / (k + 1)) * ((2.0 * k + 1.0) * (t * p1) - (double)k * p0);
    const cplx d2 = d0 + (2.0 * k + 1.0) * p1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    for (int c = 0; c < 3; ++c) {
      const double ck = coef[(k + 1) * stride + c];
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

}  // namespace rrq
