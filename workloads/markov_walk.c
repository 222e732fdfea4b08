/* Walk of an order-`order` Markov chain for the synthetic workloads: the
 * next symbol is perms[context][rank[t]], context = the previous `order`
 * symbols in base k.  All randomness (start symbols, ranks, permutations) is
 * drawn by the caller; this loop only applies the recurrence. */
#include <stdint.h>

void markov_walk(int64_t n, int order, int k, const int64_t *perms,
                 const uint8_t *ranks /* n - order */, uint8_t *sym /* n, first `order` preset */) {
  int64_t kk = 1;
  for (int d = 0; d < order; d++) kk *= k;
  int64_t ctx = 0;
  for (int64_t t = 0; t < order && t < n; t++) ctx = (ctx * k + sym[t]) % kk;
  for (int64_t t = order; t < n; t++) {
    uint8_t x = (uint8_t)perms[ctx * k + ranks[t - order]];
    sym[t] = x;
    ctx = (ctx * k + x) % kk;
  }
}
