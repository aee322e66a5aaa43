// Host check of the activation rule's sin_cos (act_math.h) against FP64 sin
// and cos: every quadrant, both signs, arguments up to the stated bound.
// Prints the worst absolute errors.
#include <cmath>
#include <cstdio>
#include <random>

#include "../../paper_2104_10013_amd/csrc/act_math.h"

int main() {
  double worst_s = 0.0, worst_c = 0.0, worst_s_small = 0.0, worst_c_small = 0.0;
  long n = 0;
  std::mt19937_64 rng(12345);
  auto check = [&](float y) {
    float s, c;
    ddp::sin_cos(y, s, c);
    const double es = std::fabs((double)s - std::sin((double)y));
    const double ec = std::fabs((double)c - std::cos((double)y));
    worst_s = std::fmax(worst_s, es);
    worst_c = std::fmax(worst_c, ec);
    if (std::fabs(y) <= 100.f) {
      worst_s_small = std::fmax(worst_s_small, es);
      worst_c_small = std::fmax(worst_c_small, ec);
    }
    ++n;
  };
  // a dense sweep of [-8 pi, 8 pi] (all four quadrants, several periods)
  for (int i = -2000000; i <= 2000000; ++i) check((float)(i * (8.0 * M_PI / 2000000.0)));
  // quadrant boundaries and their float neighbours
  for (int k = -64; k <= 64; ++k) {
    const float b = (float)(k * M_PI / 4.0);
    check(b);
    check(std::nextafter(b, 1e30f));
    check(std::nextafter(b, -1e30f));
  }
  // log-uniform magnitudes up to the bound, both signs
  std::uniform_real_distribution<double> ul(-6.0, std::log10((double)ddp::kSinCosMaxArg));
  for (int i = 0; i < 2000000; ++i) {
    const float y = (float)std::pow(10.0, ul(rng));
    check(y);
    check(-y);
  }
  check(ddp::kSinCosMaxArg);
  check(-ddp::kSinCosMaxArg);
  check(0.f);
  check(-0.f);
  std::printf("n %ld worst_sin %.3e worst_cos %.3e worst_sin_small %.3e worst_cos_small %.3e\n", n, worst_s,
              worst_c, worst_s_small, worst_c_small);
  return 0;
}
