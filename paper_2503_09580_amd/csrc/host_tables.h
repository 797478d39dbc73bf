// Host-side plan precomputation (FP64).  See host_tables.cpp.
#pragma once
#include <vector>

namespace lincoll {

struct TableParams {
  int n;
  double L, omega, C, R;
  int J;
  int quad_rule;
};

struct HostTables {
  int n = 0, J = 0, Q = 0;
  std::vector<double> g, W;     // [J]
  std::vector<double> Phi;      // [J][Q], Q = 3(n/2)^2 + 1, indexed by |k|^2
  std::vector<double> Omega;    // [Q]
  std::vector<double> phi;      // [J][P][P][P], P = n/2 + 1, octant of iDFT[sigma_j]
  std::vector<double> Cdct;     // [P][P], folded DFT of an even real-space kernel
};

bool build_tables(const TableParams& tp, HostTables& t);

// Positive Gauss-Legendre nodes (polar cosines) and weights of the
// n_polar-point rule (n_polar even) for the hemisphere product rule.
bool hemisphere_polar(int n_polar, std::vector<double>& mu, std::vector<double>& w);

}  // namespace lincoll
