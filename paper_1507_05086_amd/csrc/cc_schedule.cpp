// cc_schedule.cpp -- the paper's practical schedule (Implementation Details:
// "Estimating but not computing Delta" and "Binomial sampling instead of
// fixed-size batches"), drawn on the host.
//
//   Delta-hat_i = Delta_0 / 2^floor(i / K),  K = ceil((2/eps) ln(n L / delta)),
//   L = max(log2 Delta_0, 1);  p_i = min(1, eps / Delta-hat_i) (1 if Delta_0 = 0);
//   B_i ~ Binomial(N_i, p_i), N_i = pi positions not yet passed.
//
// The sequence B_0, B_1, ... depends on (n, Delta_0, eps, delta, seed) only,
// never on which vertices are clustered, so it is drawn once before the
// round loop (one variate per round, microseconds in all) and the device
// reads it like a replayed schedule.  Drawing it on the host keeps the
// library and any other implementation of the same published steps in exact
// agreement: both use IEEE double arithmetic as written (contraction off) and
// the host C library's log, pow and lgamma.
//
// Variates: round i uses the uniforms (x >> 11) 2^-53 of SplitMix64 (Steele,
// Lea, Flood 2014) outputs number i 2^32 + k, k = 0, 1, ...; Binomial(N, p)
// = N - Binomial(N, 1 - p) for p > 1/2, else sequential-search inversion
// (Kachitvichyanukul and Schmeiser's BINV, 1988) for N p < 10, else
// Hormann's transformed rejection with decomposition (BTRD, 1993).
#include <cmath>
#include <cstdint>
#include <vector>

#include "cc_schedule.h"

// every floating-point step rounds as written: no fused multiply-add
#pragma clang fp contract(off)

namespace ccd {
namespace {

class Uniforms {
 public:
  Uniforms(uint64_t seed, uint64_t round) : key_(seed), next_(round << 32) {}
  double operator()() {
    uint64_t z = key_ + (next_ + 1) * 0x9E3779B97F4A7C15ULL;  // SplitMix64 output number next_
    ++next_;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return static_cast<double>(z >> 11) * 0x1.0p-53;
  }

 private:
  uint64_t key_, next_;
};

// P(0) = q^N, P(x) = P(x-1) ((N+1) p/q / x - p/q); the first x at which the
// running sum passes u.  A walk past N (rounding in the far tail) redraws.
int64_t inversion(int64_t n, double p, Uniforms &u01) {
  const double q = 1.0 - p;
  const double odds = p / q;
  const double scaled = static_cast<double>(n + 1) * odds;
  const double p0 = std::pow(q, static_cast<double>(n));
  for (;;) {
    double u = u01();
    double pk = p0;
    int64_t x = 0;
    bool past_end = false;
    while (u > pk) {
      u -= pk;
      if (++x > n) {
        past_end = true;
        break;
      }
      pk *= scaled / static_cast<double>(x) - odds;
    }
    if (!past_end) return x;
  }
}

// log k! minus Stirling's (k + 1/2) log(k+1) - (k+1) + log(2 pi)/2: exact
// below 10, else the first three terms of its series in 1/(k+1).
double stirling_rest(int64_t k) {
  const double x = static_cast<double>(k) + 1.0;
  if (k <= 9) return std::lgamma(x) - (static_cast<double>(k) + 0.5) * std::log(x) + x - 0.91893853320467274178;
  const double x2 = x * x;
  return (1.0 / 12.0 - (1.0 / 360.0 - 1.0 / 1260.0 / x2) / x2) / x;
}

// BTRD for N p >= 10, p <= 1/2 (mode m).
int64_t transformed_rejection(int64_t n, double p, Uniforms &u01) {
  const double q = 1.0 - p;
  const double npq = static_cast<double>(n) * p * q;
  const double spq = std::sqrt(npq);
  const double b = 1.15 + 2.53 * spq;
  const double a = -0.0873 + 0.0248 * b + 0.01 * p;
  const double c = static_cast<double>(n) * p + 0.5;
  const double alpha = (2.83 + 5.1 / b) * spq;
  const double vr = 0.92 - 4.2 / b;
  const double urvr = 0.86 * vr;
  const int64_t m = static_cast<int64_t>(std::floor(static_cast<double>(n + 1) * p));
  const double r = p / q;
  const double nr = static_cast<double>(n + 1) * r;
  for (;;) {
    double v = u01();
    double u;
    if (v <= urvr) {  // the hat's centre: accept at once
      u = v / vr - 0.43;
      return static_cast<int64_t>(std::floor((2.0 * a / (0.5 - std::fabs(u)) + b) * u + c));
    }
    if (v >= vr) {
      u = u01() - 0.5;
    } else {
      u = v / vr - 0.93;
      u = (u < 0.0 ? -0.5 : 0.5) - u;
      v = u01() * vr;
    }
    const double us = 0.5 - std::fabs(u);
    const double kf = std::floor((2.0 * a / us + b) * u + c);
    if (kf < 0.0 || kf > static_cast<double>(n)) continue;
    const int64_t k = static_cast<int64_t>(kf);
    v = v * alpha / (a / (us * us) + b);
    const int64_t km = k > m ? k - m : m - k;
    if (km <= 15) {  // f(k) / f(m) as a product of successive ratios
      double f = 1.0;
      if (m < k) {
        for (int64_t i = m + 1; i <= k; i++) f *= nr / static_cast<double>(i) - r;
      } else if (m > k) {
        for (int64_t i = k + 1; i <= m; i++) v *= nr / static_cast<double>(i) - r;
      }
      if (v <= f) return k;
      continue;
    }
    v = std::log(v);  // squeeze on log f(k) / f(m)
    const double dkm = static_cast<double>(km);
    const double rho = (dkm / npq) * (((dkm / 3.0 + 0.625) * dkm + 1.0 / 6.0) / npq + 0.5);
    const double t = -dkm * dkm / (2.0 * npq);
    if (v < t - rho) return k;
    if (v > t + rho) continue;
    const double nm = static_cast<double>(n - m + 1);
    const double h = (static_cast<double>(m) + 0.5) * std::log((static_cast<double>(m) + 1.0) / (r * nm)) +
                     stirling_rest(m) + stirling_rest(n - m);
    const double nk = static_cast<double>(n - k + 1);
    if (v <= h + static_cast<double>(n + 1) * std::log(nm / nk) +
                 (static_cast<double>(k) + 0.5) * std::log(nk * r / (static_cast<double>(k) + 1.0)) -
                 stirling_rest(k) - stirling_rest(n - k))
      return k;
  }
}

int64_t draw_binomial(uint64_t seed, uint64_t round, int64_t n, double p) {
  if (n <= 0 || p <= 0.0) return 0;
  if (p >= 1.0) return n;
  Uniforms u01(seed, round);
  if (p > 0.5) {
    const double pc = 1.0 - p;
    return n - (static_cast<double>(n) * pc < 10.0 ? inversion(n, pc, u01) : transformed_rejection(n, pc, u01));
  }
  return static_cast<double>(n) * p < 10.0 ? inversion(n, p, u01) : transformed_rejection(n, p, u01);
}

double sample_probability(int64_t round, int64_t period, int64_t delta0, double eps) {
  if (delta0 <= 0) return 1.0;
  const int64_t halvings = round / period;
  if (halvings > 1000) return 1.0;
  const double pr = std::ldexp(eps / static_cast<double>(delta0), static_cast<int>(halvings));
  return pr < 1.0 ? pr : 1.0;
}

}  // namespace

int64_t halving_period(int64_t n, int64_t delta0, double eps, double delta) {
  double lg = delta0 > 1 ? std::log2(static_cast<double>(delta0)) : 1.0;
  if (lg < 1.0) lg = 1.0;
  const double arg = static_cast<double>(n > 1 ? n : 1) * lg / delta;
  const double k = std::ceil(2.0 / eps * std::log(arg));
  return k < 1.0 ? 1 : static_cast<int64_t>(k);
}

void binomial_schedule(int64_t n, int64_t delta0, double eps, double delta, uint64_t seed,
                       std::vector<int64_t> *out) {
  out->clear();
  const int64_t period = halving_period(n, delta0, eps, delta);
  int64_t left = n;
  for (int64_t i = 0; left > 0; i++) {
    const int64_t b = draw_binomial(seed, static_cast<uint64_t>(i), left,
                                    sample_probability(i, period, delta0, eps));
    out->push_back(b);
    left -= b;
  }
}

}  // namespace ccd
