// Host check of the reverse-mode VJP of the TTP06 currents (ttp06_vjp.h)
// against central differences of ttp06::currents, both run on the host.
// Input (stdin): n, then n lines of 19 states; cotangents and scalings are
// drawn here.  Output: the largest relative deviation over states and inputs.
#include <cmath>
#include <cstdio>
#include <random>

#include "ttp06_vjp.h"

static double objective(const double *y, const double *gs, double cI, const double *ch) {
  double I, ha[6];
  ttp06::currents<double>(y, gs[0], gs[1], gs[2], I, ha);
  double v = cI * I;
  for (int k = 0; k < 6; ++k) v += ch[k] * ha[k];
  return v;
}

int main() {
  int n = 0;
  if (std::scanf("%d", &n) != 1 || n <= 0) return 2;
  std::mt19937_64 rng(7);
  std::uniform_real_distribution<double> U(-1.0, 1.0), G(0.8, 1.2);
  double worst = 0.0;
  for (int q = 0; q < n; ++q) {
    double y[19];
    for (int k = 0; k < 19; ++k)
      if (std::scanf("%lf", &y[k]) != 1) return 2;
    const double gs[3] = {G(rng), G(rng), G(rng)};
    const double cI = U(rng);
    double ch[6];
    for (double &c : ch) c = U(rng);
    double vx[19] = {0}, vgs[3] = {0};
    ttp06::currents_vjp<double>(y, gs[0], gs[1], gs[2], cI, ch, vx, vgs);
    for (int k = 0; k < 22; ++k) {
      double yp[19], ym[19], gp[3], gm[3];
      for (int f = 0; f < 19; ++f) yp[f] = ym[f] = y[f];
      for (int f = 0; f < 3; ++f) gp[f] = gm[f] = gs[f];
      double hstep;
      if (k < 19) {
        hstep = 1e-6 * std::fmax(std::fabs(y[k]), 1e-6);
        yp[k] += hstep;
        ym[k] -= hstep;
      } else {
        hstep = 1e-6;
        gp[k - 19] += hstep;
        gm[k - 19] -= hstep;
      }
      const double fd = (objective(yp, gp, cI, ch) - objective(ym, gm, cI, ch)) / (2.0 * hstep);
      const double an = k < 19 ? vx[k] : vgs[k - 19];
      // relative to the derivative's own size, floored by the objective's
      // sensitivity scale (rounding of the differences)
      const double scale = std::fabs(fd) + std::fabs(an) +
                           1e-9 * std::fabs(objective(y, gs, cI, ch)) / hstep;
      const double rel = std::fabs(an - fd) / scale;
      if (rel > worst) worst = rel;
      if (rel > 1e-5) std::printf("state %d input %d: vjp %.10e fd %.10e\n", q, k, an, fd);
    }
  }
  std::printf("worst %.3e\n", worst);
  return worst < 1e-5 ? 0 : 1;
}
