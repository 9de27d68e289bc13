// cc_schedule.h -- host side of the practical schedule (Delta-hat halving and
// Binomial batches over pi positions); see cc_schedule.cpp.
#pragma once
#include <cstdint>
#include <vector>

namespace ccd {

// K: rounds between two halvings of Delta-hat, ceil((2/eps) ln(n L / delta)).
int64_t halving_period(int64_t n, int64_t delta0, double eps, double delta);

// B_0, B_1, ... until the n positions are used up.
void binomial_schedule(int64_t n, int64_t delta0, double eps, double delta, uint64_t seed,
                       std::vector<int64_t> *out);

}  // namespace ccd
