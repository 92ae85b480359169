// Structural check of the translation slot tables built on the host (rrq_consts.cpp): for
// every supported order, the pieces of each (l, m) term list partition it in order, the pieces
// of a list sit on adjacent slots starting at a multiple of their count, the packed operand
// offsets and the coefficients of every piece match the merged list term by term, chunk tails
// and the read-ahead row are zero, and the slots of 4 targets fit the chosen passes.
// Prints one line per order; exit status 1 on the first violation.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_2411_08342_amd/csrc/rrq_consts.h"

using namespace rrq;

static int fail(int q, const char* what, int a, int b) {
  std::printf("FAIL q=%d %s (%d, %d)\n", q, what, a, b);
  return 1;
}

int main() {
  for (int q : {4, 5, 6, 8, 10}) {
    const OrderTables T = build_order_tables(q, 2 * q);
    const int ns = (int)T.tslot.size();
    if (ns % 4) return fail(q, "slot count not a multiple of 4", ns, 0);
    std::vector<int> next(T.np, 0);   // next expected piece of each list
    int maxlen = 0;
    for (int sl = 0; sl < ns; ++sl) {
      const int code = T.tslot[sl];
      const int len = T.tlen[sl];
      maxlen = len > maxlen ? len : maxlen;
      if (code == kPadSlot) {
        if (len != 0) return fail(q, "padding slot with terms", sl, len);
        continue;
      }
      const int lm = code & 0xff, pc = (code >> 8) & 0xf, lg = code >> 12, g = 1 << lg;
      if (lg > 2 || pc >= g) return fail(q, "bad piece code", sl, code);
      if ((sl - pc) % g) return fail(q, "piece group not aligned", sl, g);
      if (pc != next[lm]) return fail(q, "pieces out of order", sl, pc);
      next[lm] = pc + 1;
      const int it0 = T.mrg_ptr[lm], n = T.mrg_ptr[lm + 1] - it0;
      const int b0 = it0 + n * pc / g, b1 = it0 + n * (pc + 1) / g;
      if (len != b1 - b0) return fail(q, "piece length", sl, len);
      for (int i = 0; i < T.tchunks * kTermChunk; ++i) {
        const int32_t nr = T.tnr[((size_t)(i / kTermChunk) * ns + sl) * kTermChunk + i % kTermChunk];
        const double* cf = &T.tcf[4 * ((size_t)i * ns + sl)];
        if (i < len) {
          const Term2& t = T.mrg[b0 + i];
          if (nr != (vq_rec(t.n) << 8 | t.r)) return fail(q, "packed offsets", sl, i);
          if (cf[0] != t.cDr || cf[1] != t.cDi || cf[2] != t.cSr || cf[3] != t.cSi)
            return fail(q, "coefficients", sl, i);
        } else if (nr != 0 || cf[0] != 0.0 || cf[1] != 0.0 || cf[2] != 0.0 || cf[3] != 0.0) {
          return fail(q, "chunk tail not zero", sl, i);
        }
      }
    }
    for (int lm = 0; lm < T.np; ++lm) {
      const int n = T.mrg_ptr[lm + 1] - T.mrg_ptr[lm];
      if (n <= 0) return fail(q, "empty or flagged term list", lm, n);
      if (next[lm] != 1 && next[lm] != 2 && next[lm] != 4) return fail(q, "list pieces", lm, next[lm]);
    }
    for (int sl = 0; sl < ns; ++sl)
      for (int u = 0; u < kTermChunk; ++u)
        if (T.tnr[((size_t)T.tchunks * ns + sl) * kTermChunk + u] != 0)
          return fail(q, "read-ahead row not zero", sl, u);
    if (T.tsteps != maxlen || T.tchunks != (maxlen + kTermChunk - 1) / kTermChunk)
      return fail(q, "tsteps/tchunks", T.tsteps, T.tchunks);
    std::printf("q=%d lists=%d terms=%zu slots=%d longest=%d chunks=%d passes_T4=%d\n", q, T.np,
                T.mrg.size(), ns, maxlen, T.tchunks, (4 * ns + 255) / 256);
  }
  return 0;
}
