// Constant tables (host, long double): Gauss-Legendre rules, the inverse Vandermonde matrix U
// of the edge interpolation (Sec. 3.5) and the index/coefficient lists of the translation
// sums of eq. cdlp1dintegral and Theorem thm:cslp1form.
#include "rrq_consts.h"

#include <math.h>

#include <algorithm>

namespace rrq {

void gauss_legendre_ld(int n, std::vector<double>& t, std::vector<double>& w) {
  t.assign(n, 0.0);
  w.assign(n, 0.0);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    long double x = cosl(pi * (i + 0.75L) / (n + 0.5L));
    long double dp = 0;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = x;
      for (int k = 2; k <= n; ++k) {
        long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = x; p0 = 1; }
      dp = n * (x * p1 - p0) / (x * x - 1);
      long double dx = p1 / dp;
      x -= dx;
      if (fabsl(dx) < 1e-19L) break;
    }
    long double p0 = 1, p1 = x;
    for (int k = 2; k <= n; ++k) {
      long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (x * p1 - p0) / (x * x - 1);
    t[n - 1 - i] = (double)x;                       // increasing order
    w[n - 1 - i] = (double)(2.0L / ((1 - x * x) * dp * dp));
  }
}

static long double binom_ld(int n, int k) {
  if (k < 0 || k > n || n < 0) return 0;
  long double r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

static long double fact_ld(int n) {
  long double r = 1;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}

OrderTables build_order_tables(int q, int pt) {
  OrderTables T;
  T.q = q;
  T.pt = pt;
  T.np = np_of(q);
  T.njk = njk_of(q);
  gauss_legendre_ld(pt, T.gl_t, T.gl_w);
  std::vector<double> tq;
  gauss_legendre_ld(q, tq, T.glq_w);

  // U = V^{-1}, V[i][k] = t_i^k, by Gauss-Jordan elimination in long double
  std::vector<long double> A(pt * 2 * pt, 0.0L);
  for (int i = 0; i < pt; ++i) {
    long double x = T.gl_t[i], p = 1;
    for (int k = 0; k < pt; ++k) {
      A[i * 2 * pt + k] = p;
      p *= x;
    }
    A[i * 2 * pt + pt + i] = 1;
  }
  for (int c = 0; c < pt; ++c) {
    int piv = c;
    for (int r = c + 1; r < pt; ++r)
      if (fabsl(A[r * 2 * pt + c]) > fabsl(A[piv * 2 * pt + c])) piv = r;
    if (piv != c)
      for (int k = 0; k < 2 * pt; ++k) std::swap(A[c * 2 * pt + k], A[piv * 2 * pt + k]);
    long double d = A[c * 2 * pt + c];
    for (int k = 0; k < 2 * pt; ++k) A[c * 2 * pt + k] /= d;
    for (int r = 0; r < pt; ++r) {
      if (r == c) continue;
      long double f = A[r * 2 * pt + c];
      if (f == 0) continue;
      for (int k = 0; k < 2 * pt; ++k) A[r * 2 * pt + k] -= f * A[c * 2 * pt + k];
    }
  }
  // inverse V^{-1}[k][i]: coefficient k of the Lagrange polynomial l_i
  T.U.assign(pt * pt, 0.0);
  T.lag_m1.assign(pt, 0.0);
  for (int k = 0; k < pt; ++k)
    for (int i = 0; i < pt; ++i) T.U[k * pt + i] = (double)A[k * 2 * pt + pt + i];
  for (int i = 0; i < pt; ++i) {
    long double s = 0, p = 1;
    for (int k = 0; k < pt; ++k) {
      s += A[k * 2 * pt + pt + i] * p;
      p *= -1;
    }
    T.lag_m1[i] = (double)s;
  }

  // discrete Legendre transform of the GL samples and Legendre derivatives at the nodes
  T.LT.assign(pt * pt, 0.0);
  T.DP.assign(pt * pt, 0.0);
  for (int i = 0; i < pt; ++i) {
    long double x = T.gl_t[i], p0 = 0, p1 = 1, d0 = 0, d1 = 0;
    for (int k = 0; k < pt; ++k) {
      T.LT[k * pt + i] = (double)((2 * k + 1) / 2.0L * (long double)T.gl_w[i] * p1);
      T.DP[i * pt + k] = (double)d1;
      long double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
      long double d2 = d0 + (2 * k + 1) * p1;
      p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
  }
  T.bary.assign(pt, 0.0);
  for (int i = 0; i < pt; ++i) {
    long double ti = T.gl_t[i];
    T.bary[i] = (double)((i & 1 ? -1.0L : 1.0L) * sqrtl((1 - ti * ti) * (long double)T.gl_w[i]));
  }
  // first barycentric form: l_i(t) = ell(t) bary1_i / (t - t_i), ell(t) = prod_j (t - t_j)
  T.bary1.assign(pt, 0.0);
  for (int i = 0; i < pt; ++i) {
    long double pr = 1.0L;
    for (int j = 0; j < pt; ++j)
      if (j != i) pr *= (long double)T.gl_t[i] - (long double)T.gl_t[j];
    T.bary1[i] = (double)(1.0L / pr);
  }

  // translation terms, grouped by basis function (l, m), 1 <= m <= l <= q
  T.dlp_ptr.assign(1, 0);
  T.slp_ptr.assign(1, 0);
  for (int l = 1; l <= q; ++l)
    for (int m = 1; m <= l; ++m) {
      for (int pass = 0; pass < 2; ++pass) {
        const int j0 = pass == 0 ? 2 : 1;
        for (int j = j0; j <= l; ++j) {
          long double wj = pass == 0
                               ? fact_ld(j - 2) * fact_ld(l - j) / fact_ld(l - 1)   // C_{j,l}
                               : fact_ld(j - 1) * fact_ld(l - j) / fact_ld(l);      // D_{j,l}
          for (int k = -j; k <= j; ++k) {
            if (std::abs(m - k) > l - j) continue;
            long double tc = sqrtl(binom_ld(l + m, j + k) * binom_ld(l - m, j - k));
            Term t;
            int ak = std::abs(k);
            t.n = jk_index(j, ak);
            t.a = (int16_t)(l - j);
            t.b = (int16_t)(m - k);
            t.neg = k < 0;
            long double sg = (k < 0 && (ak & 1)) ? -1.0L : 1.0L;
            t.coef = (double)(wj * tc * sg);
            (pass == 0 ? T.dlp : T.slp).push_back(t);
          }
        }
        (pass == 0 ? T.dlp_ptr : T.slp_ptr).push_back(
            (int32_t)(pass == 0 ? T.dlp.size() : T.slp.size()));
      }
    }
  // merged lists: the double-layer terms are the single-layer terms with j >= 2, in the same
  // (j, k) order
  T.mrg_ptr.assign(1, 0);
  for (int lm = 0; lm < T.np; ++lm) {
    int d = T.dlp_ptr[lm];
    for (int s = T.slp_ptr[lm]; s < T.slp_ptr[lm + 1]; ++s) {
      const Term& ts = T.slp[s];
      double cD = 0.0;
      if (d < T.dlp_ptr[lm + 1] && T.dlp[d].n == ts.n && T.dlp[d].a == ts.a &&
          T.dlp[d].b == ts.b && T.dlp[d].neg == ts.neg) {
        cD = T.dlp[d].coef;
        ++d;
      }
      const int ab = std::abs((int)ts.b);
      const double sr = (ts.b < 0 && (ab & 1)) ? -1.0 : 1.0;
      const double si = (ts.b < 0 && !(ab & 1)) ? -1.0 : 1.0;
      const double nu = ts.neg ? -1.0 : 1.0;
      Term2 t2;
      t2.n = ts.n;
      t2.r = ts.a * (ts.a + 1) / 2 + ab;
      t2.cDr = cD * sr * nu;
      t2.cDi = cD * si;
      t2.cSr = ts.coef * sr * nu;
      t2.cSi = ts.coef * si;
      T.mrg.push_back(t2);
    }
    T.mrg_ptr.push_back((int32_t)T.mrg.size());
    if (d != T.dlp_ptr[lm + 1]) T.mrg_ptr.back() = -1;   // not a subset: flagged for the caller
  }
  // translation slots: the term list of each (l, m) is split evenly into g = 1, 2 or 4
  // pieces, one slot each; the g slots of a list are adjacent and start at a multiple of g.
  // The bound M on a piece's length (a multiple of the chunk) is the one for which the slots
  // of 4 targets take the fewest passes of a 256-lane workgroup times chunks per piece (ties:
  // fewer slots).  The slot count is a multiple of 4, so that a list's pieces sit on lanes of
  // one aligned group of the wavefront whichever target they belong to.
  auto pieces = [&](int len, int M) {
    int g = 1;
    while ((len + g - 1) / g > M && g < 4) g *= 2;
    return (len + g - 1) / g > M ? 0 : g;
  };
  int bestM = 0;
  long best_cost = 0, best_n = 0;
  for (int M = kTermChunk; M <= 1024; M += kTermChunk) {
    long n = 0;
    bool ok = true;
    for (int lm = 0; lm < T.np && ok; ++lm) {
      const int g = pieces(T.mrg_ptr[lm + 1] - T.mrg_ptr[lm], M);
      ok = g > 0;
      n += g;
    }
    if (!ok) continue;
    n += (4 - n % 4) % 4;
    const long cost = ((4 * n + 255) / 256) * (M / kTermChunk);
    if (bestM == 0 || cost < best_cost || (cost == best_cost && n < best_n)) {
      bestM = M;
      best_cost = cost;
      best_n = n;
    }
  }
  std::vector<int> tbeg, tend;
  for (int lg = 2; lg >= 0; --lg)   // groups of 4 first, then pairs, then single lists
    for (int lm = 0; lm < T.np; ++lm) {
      const int it0 = T.mrg_ptr[lm], len = T.mrg_ptr[lm + 1] - it0;
      const int g = pieces(len, bestM);
      if (g != 1 << lg) continue;
      for (int pc = 0; pc < g; ++pc) {
        T.tslot.push_back(lm | pc << 8 | lg << 12);
        tbeg.push_back(it0 + len * pc / g);
        tend.push_back(it0 + len * (pc + 1) / g);
      }
    }
  while (T.tslot.size() % 4) {
    T.tslot.push_back(kPadSlot);
    tbeg.push_back(0);
    tend.push_back(0);
  }
  const int ns = (int)T.tslot.size();
  T.tlen.assign(ns, 0);
  for (int sl = 0; sl < ns; ++sl) {
    T.tlen[sl] = tend[sl] - tbeg[sl];
    T.tsteps = std::max(T.tsteps, T.tlen[sl]);
  }
  for (int sl = 0; sl < ns; ++sl)
    T.tchunks = std::max(T.tchunks, (T.tlen[sl] + kTermChunk - 1) / kTermChunk);
  const int npad = T.tchunks * kTermChunk;
  T.tnr.assign((size_t)(T.tchunks + 1) * ns * kTermChunk, 0);
  T.tcf.assign((size_t)npad * ns * 4, 0.0);
  for (int sl = 0; sl < ns; ++sl)
    for (int i = 0; i < T.tlen[sl]; ++i) {
      const Term2& t2 = T.mrg[tbeg[sl] + i];
      T.tnr[((size_t)(i / kTermChunk) * ns + sl) * kTermChunk + i % kTermChunk] =
          vq_rec(t2.n) << 8 | t2.r;
      const size_t e = (size_t)i * ns + sl;
      T.tcf[4 * e] = t2.cDr;
      T.tcf[4 * e + 1] = t2.cDi;
      T.tcf[4 * e + 2] = t2.cSr;
      T.tcf[4 * e + 3] = t2.cSi;
    }
  return T;
}

}  // namespace rrq
