// Test driver of the host eigensolver: reads d and a row-major d x d matrix
// from stdin, prints "ok" or "fail", then the eigenvalues and the
// eigenvectors (one per line, in the solver's order).
#include <cstdio>
#include <vector>

#include "../../paper_2204_08988_amd/csrc/eigen.hpp"

int main() {
  int d = 0;
  if (std::scanf("%d", &d) != 1 || d < 1) return 2;
  std::vector<double> A((size_t)d * d), w, V;
  for (auto& a : A)
    if (std::scanf("%lf", &a) != 1) return 2;
  const bool ok = dpmm::eig::sym_eigen(A, d, w, V);
  std::printf("%s\n", ok ? "ok" : "fail");
  for (int i = 0; i < d; ++i) std::printf("%.17g ", w[i]);
  std::printf("\n");
  for (int j = 0; j < d; ++j) {
    for (int i = 0; i < d; ++i) std::printf("%.17g ", V[(size_t)j * d + i]);
    std::printf("\n");
  }
  return 0;
}
