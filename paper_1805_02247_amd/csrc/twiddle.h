// Twiddle factors exp(-2 pi i j / n), j < n, of the FFT kernels, evaluated at compile time:
// exact quadrant reduction in integers, then Taylor series of cos and sin on [0, pi/2] in
// double precision (terms to x^41 / 41!, below 1e-20), rounded once to float. The tables sit
// in device memory; a workgroup copies the one it needs into LDS instead of evaluating
// transcendentals.
#pragma once

namespace pmr {

struct TwEntry {
  float re, im;
};

template <int N>
struct TwTable {
  TwEntry v[N];
};

constexpr double kTwoPiOver4 = 1.57079632679489661923132169163975144;  // pi / 2

constexpr double taylor_sin(double x) {
  const double x2 = x * x;
  double term = x, sum = x;
  for (int k = 1; k <= 20; ++k) {
    term *= -x2 / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}

constexpr double taylor_cos(double x) {
  const double x2 = x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k <= 20; ++k) {
    term *= -x2 / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

// cos and sin of 2 pi j / n for 0 <= j < n.
constexpr void cos_sin_turn(long j, long n, double& c, double& s) {
  const long q = (4 * j) / n;        // quadrant
  const long rem = 4 * j - q * n;    // 0 <= rem < n
  const double t = kTwoPiOver4 * ((double)rem / (double)n);
  const double C = taylor_cos(t), S = taylor_sin(t);
  switch (q) {
    case 0: c = C; s = S; break;
    case 1: c = -S; s = C; break;
    case 2: c = -C; s = -S; break;
    default: c = S; s = -C; break;
  }
}

template <int N>
constexpr TwTable<N> make_tw_table() {
  TwTable<N> t{};
  for (int j = 0; j < N; ++j) {
    double c = 0.0, s = 0.0;
    cos_sin_turn(j, N, c, s);
    t.v[j] = TwEntry{(float)c, (float)(-s)};
  }
  return t;
}

}  // namespace pmr
