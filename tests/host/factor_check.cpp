// Host check of the step-1 factorisation (factor_K in the library's host
// setup code): for random sparse constraint matrices A (m rows over nE
// entries) and positive weights p, K = shift I + A diag(p) A^T is factorised
// and K^{-1} applied to g = K x, with g formed from the definition
// (shift x + A (p o (A^T x))); prints the relative error ||x - K^{-1} g|| /
// ||x|| and whether the dense or the sparse form was taken.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_1611_01828_amd/csrc/plan.h"

int main(int argc, char** argv) {
  if (argc < 6) return 2;
  const int m = std::atoi(argv[1]), nE = std::atoi(argv[2]), per_row = std::atoi(argv[3]);
  const double shift = std::atof(argv[4]);
  const unsigned seed = (unsigned)std::atoi(argv[5]);
  std::mt19937_64 gen(seed);
  std::uniform_int_distribution<int> col(0, nE - 1);
  std::normal_distribution<double> nrm(0.0, 1.0);
  std::uniform_real_distribution<double> pos(0.2, 1.0);
  std::vector<int32_t> aptr(m + 1, 0), acol;
  std::vector<double> aval;
  for (int i = 0; i < m; ++i) {
    std::vector<int32_t> cs;
    // one entry of its own per row (full row rank for shift 0), then random ones
    cs.push_back((int32_t)((long)i * nE / m));
    while ((int)cs.size() < per_row) cs.push_back(col(gen));
    std::sort(cs.begin(), cs.end());
    cs.erase(std::unique(cs.begin(), cs.end()), cs.end());
    for (int32_t c : cs) {
      acol.push_back(c);
      aval.push_back(nrm(gen));
    }
    aptr[i + 1] = (int32_t)acol.size();
  }
  std::vector<double> p(nE);
  for (auto& v : p) v = pos(gen);
  cdcs::Factor f;
  cdcs::Error err{0, ""};
  const int rc = cdcs::factor_K(m, aptr, acol, aval, p, f, err, shift);
  if (rc) {
    std::printf("error %d %s\n", rc, err.msg.c_str());
    return 1;
  }
  std::vector<double> x(m), g(m), at(nE, 0.0);
  for (auto& v : x) v = nrm(gen);
  for (int i = 0; i < m; ++i)
    for (int q = aptr[i]; q < aptr[i + 1]; ++q) at[acol[q]] += aval[q] * x[i];
  for (int i = 0; i < m; ++i) {
    double s = shift * x[i];
    for (int q = aptr[i]; q < aptr[i + 1]; ++q) s += aval[q] * p[acol[q]] * at[acol[q]];
    g[i] = s;
  }
  f.solve(g);
  double num = 0.0, den = 0.0;
  for (int i = 0; i < m; ++i) {
    num += (g[i] - x[i]) * (g[i] - x[i]);
    den += x[i] * x[i];
  }
  std::printf("%s %.3e\n", f.dense ? "dense" : "sparse", std::sqrt(num / den));
  return 0;
}
