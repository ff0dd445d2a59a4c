// exact_rule.h -- which entries of a (sample, SNR) item the exact path
// recomputes. Plain C++ (a constexpr function, usable in device code), so that
// host tests can check the rule itself.
#pragma once
#include <stdint.h>

namespace air {

// An item's fast-path sums: the total over all points and side[2k + b], the
// sum over bit side (k, b), k < m. An entry below thr (or NaN) is starved.
// When the total is starved, every side is recomputed, since all of them are
// then taken relative to the nearest point: a side is not below the total bit
// for bit (the two are summed in different orders), so a side can sit above
// thr while the total is below it. Otherwise only the starved sides are
// recomputed. Bit i of the result is side entry i.
template <typename T>
constexpr uint32_t exact_entries(T total, const T* side, int m, T thr) {
  const bool total_slow = !(total >= thr);
  uint32_t mask = 0;
  for (int i = 0; i < 2 * m; ++i)
    if (total_slow || !(side[i] >= thr)) mask |= 1u << i;
  return mask;
}

}  // namespace air
