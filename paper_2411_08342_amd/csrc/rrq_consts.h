// Host-side constant tables of the quadrature rules and of the translation sums.
// Computed once per order in extended precision and uploaded with the plan.
#pragma once
#include <stdint.h>

#include <vector>

namespace rrq {

constexpr int kMaxQ = 10;
constexpr int kNumOrders = 5;
constexpr int kOrders[kNumOrders] = {4, 5, 6, 8, 10};

__host__ __device__ constexpr int np_of(int p) { return p * (p + 1) / 2; }
__host__ __device__ constexpr int njk_of(int p) { return p * (p + 3) / 2; }   // (j,k), 1<=j<=p, 0<=k<=j
__host__ __device__ constexpr int jk_index(int j, int k) { return j * (j + 1) / 2 - 1 + k; }
// LDS offset (doubles) of the 18 moments of (j,k) index n within a target's block: one spare
// double after every 8 records, so that 8-byte reads of lane-scattered records fall on all 32
// banks (the record stride alone, 36 dwords, reaches only every fourth bank)
__host__ __device__ constexpr int vq_rec(int n) { return 18 * n + (n >> 3); }

// one term of a translation sum: out[lm] += coef * X^{(j,|k|)} (conj if neg) * S^{(a,b)}(x)
struct Term {
  int32_t n;      // index of (j, |k|) in the jk table
  int16_t a, b;   // S^{(a,b)}: a = l - j, b = m - k (b may be negative)
  int32_t neg;    // k < 0: use conj(X^{(j,|k|)})
  double coef;    // (weight C_{j,l} or D_{j,l}) * T_{jk,lm} * (-1)^{|k|} if k < 0
};

// one term of the merged translation sum over the (j, k) index set of the single-layer sum;
// the double-layer weight (cDr, cDi) is zero for j = 1.  Only imaginary parts of the sums
// are used (eq. wlmdef takes Im), so a term contributes Im(X' c S') with X' = X^{(j,|k|)},
// conjugated for k < 0, and S' = S^{(a,b)} = +-S^{(a,|b|)} or its conjugate for b < 0
// (rget).  Both sign patterns are folded into the weights: with s = S^{(a,|b|)},
//   Im(X' c S') = X.re (c_i s.im) + X.im (c_r s.re),  c_i = c sigma_i, c_r = c sigma_r nu,
// nu = -1 for k < 0, (sigma_r, sigma_i) = (1, 1) for b >= 0, (-1, 1) for odd b < 0,
// (1, -1) for even b < 0.  Every sign is exact, so the sums round as the unfolded form.
struct Term2 {
  int32_t n;      // index of (j, |k|) in the jk table
  int32_t r;      // index tri(a, |b|) of S^{(a,|b|)} in the target tables
  double cDr, cDi;  // C_{j,l} T_{jk,lm} (sign for k < 0 included), folded as above
  double cSr, cSi;  // D_{j,l} T_{jk,lm} (sign for k < 0 included), folded as above
};

struct OrderTables {
  int q, pt, np, njk;
  std::vector<double> gl_t, gl_w;     // ptilde-point GL rule on [-1, 1]
  std::vector<double> glq_w;          // q-point GL weights (least-squares weights)
  std::vector<double> U;              // [pt][pt]: U[k*pt + i] = coeff of t^k in l_i(t)
  std::vector<double> LT;             // [pt][pt]: LT[k*pt + i] = (2k+1)/2 w_i P_k(t_i)
  std::vector<double> DP;             // [pt][pt]: DP[i*pt + k] = P_k'(t_i)
  std::vector<double> lag_m1;         // l_i(-1)
  std::vector<double> bary;           // barycentric weights (-1)^i sqrt((1 - t_i^2) w_i)
  std::vector<double> bary1;          // first-form weights 1 / prod_{j != i} (t_i - t_j)
  std::vector<int32_t> dlp_ptr, slp_ptr;   // [np+1]
  std::vector<Term> dlp, slp;
  std::vector<int32_t> mrg_ptr;        // [np+1]
  std::vector<Term2> mrg;
  // work slots of the translation step: lm | piece << 8 | lg << 12, the piece-th of the
  // 1 << lg pieces of the term list of lm (lg = 0, 1, 2; the pieces of a list sit on
  // adjacent slots starting at a multiple of 1 << lg), or kPadSlot; a multiple of 4 slots
  std::vector<int32_t> tslot;
  // the slots' term lists step-major: entry (step, slot) at step * tslot.size() + slot, so
  // that the lanes of a wavefront, one slot each, read consecutive entries at every step.
  // tlen[slot] terms per slot (0 for padding); a slot's list is processed in chunks of
  // kTermChunk steps, the last one padded with zero coefficients (operands at record 0,
  // r = 0); tchunks = the most chunks of a slot.  The operand indices of a chunk are one
  // int4, each entry vq_rec(n) << 8 | r, with one more all-zero chunk row at the end so that
  // the next chunk can always be read ahead.
  int tsteps = 0, tchunks = 0;
  std::vector<int32_t> tlen;
  std::vector<int32_t> tnr;            // [tchunks + 1][nslot][kTermChunk]: vq_rec(n) << 8 | r
  std::vector<double> tcf;             // [tchunks * kTermChunk][nslot][4]: cDr, cDi, cSr, cSi
};

void gauss_legendre_ld(int n, std::vector<double>& t, std::vector<double>& w);
constexpr int kTermChunk = 4;
constexpr int32_t kPadSlot = 3 << 12;   // a translation slot with no terms
OrderTables build_order_tables(int q, int ptilde);

}  // namespace rrq
