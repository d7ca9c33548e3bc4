// Host check of the FP32 hot word's candidacy encoding (device.h), against
// the rule the oracle applies: a particle is a collision candidate at the
// first pass k with knext <= k, and its knext is what get_state reports.
//
// For epochs E and next-pass steps k (E <= k < E + kRebaseSteps) and
// candidacies knext around the offset's range (overdue, near, at the far
// boundary, beyond, never), it checks:
//   * cell, weight class and decoded knext survive the encoding (the knext
//     array holds the step exactly when the far bit is set);
//   * stepping s = k, k+1, ... with the epoch fixed, hw_due fires at the
//     first s >= k with knext <= s and at no other s before the next
//     re-expression (s < E + kRebaseSteps + 1), or never when the
//     candidacy lies beyond that;
//   * re-expressing at a later step (as the sort does) keeps the decoded
//     knext, and a particle due before that step is due at it;
//   * hw_move changes the cell only.
// Prints "ok" and exits 0, or prints the first failing case and exits 1.
#include "device.h"

#include <cstdint>
#include <cstdio>
#include <vector>

using namespace ecpic;

static int fail(const char *what, int64_t E, int64_t k, int64_t kn) {
  std::printf("FAIL %s E=%lld k=%lld knext=%lld\n", what, (long long)E, (long long)k, (long long)kn);
  return 1;
}

int main() {
  const int64_t INT32_MAX_ = 2147483647;
  const int64_t Es[] = {0, 7, 100000, 2000000000LL - 3 * (int64_t)kCntMax};
  const int64_t gaps[] = {0, 1, 2, 999, kRebaseSteps - 1};
  int64_t checked = 0;
  for (int64_t E : Es)
    for (int64_t gap : gaps) {
      const int64_t k = E + gap;
      std::vector<int64_t> kns;
      for (int64_t d = -3; d <= 3; ++d) {
        kns.push_back(E + d);
        kns.push_back(k + d);
        kns.push_back(E + (int64_t)kCntMax + d);
        kns.push_back(E + kRebaseSteps + d);
        kns.push_back(k + kRebaseSteps + d);
      }
      kns.push_back(E + 2 * (int64_t)kCntMax + 11);
      kns.push_back(INT32_MAX_);
      for (int64_t kn : kns) {
        if (kn < 0 || kn > INT32_MAX_) continue;
        for (int cls = 0; cls < 8; cls += 3) {
          const int cell = (int)((kn * 7 + cls) % 2048);
          const uint32_t w = hw_encode(cell, kn, k, E, cls);
          const int32_t arr = hw_far(w) ? (int32_t)kn : -12345;   // the knext array
          if (!hw_live(w) || hw_cell(w) != cell || hw_class(w) != cls) return fail("fields", E, k, kn);
          if (hw_knext(w, arr, E) != kn) return fail("decode", E, k, kn);
          const bool near = kn >= k && kn - E < (int64_t)kCntMax;
          if (near == hw_far(w)) return fail("near/far", E, k, kn);
          // passes with the epoch fixed, up to the last one before a forced
          // re-expression
          const int64_t last = E + kRebaseSteps;
          const int64_t expect = kn <= k ? k : kn;   // first pass s >= k with kn <= s
          for (int64_t s = k; s <= last; ++s) {
            const bool due = hw_due(w, (uint32_t)(s - E));
            if (due != (s == expect)) return fail(due ? "due early/late" : "not due", E, s, kn);
          }
          // re-expression at a later next-pass step (a sort); a candidacy
          // that passed unqueued (collisions off) is overdue there
          for (int64_t k2 : {k + 1, k + 17, E + kRebaseSteps}) {
            if (k2 < k || k2 - E > kRebaseSteps) continue;
            const int64_t dec = hw_knext(w, arr, E);
            const uint32_t w2 = hw_encode(hw_cell(w), dec, k2, k2, hw_class(w));
            const int32_t arr2 = hw_far(w2) ? (int32_t)dec : -777;
            if (hw_knext(w2, arr2, k2) != kn) return fail("re-expressed decode", E, k2, kn);
            const bool due2 = hw_due(w2, 0u);
            if (due2 != (kn <= k2)) return fail("re-expressed due", E, k2, kn);
          }
          const uint32_t m = hw_move(w, (cell + 5) % 2048);
          if (hw_cell(m) != (cell + 5) % 2048 || (m & ~kHwCell) != (w & ~kHwCell)) return fail("move", E, k, kn);
          ++checked;
        }
      }
    }
  if (hw_live(kHwDead)) return fail("dead word", 0, 0, 0);
  std::printf("ok %lld\n", (long long)checked);
  return 0;
}
