// Host-side tables of the split-BF16x3 contraction form (orderings in mfma_layout.hpp).
#pragma once
#include <cstdint>
#include <vector>

namespace lbsmrt {

struct MfmaHostTables {
  std::vector<uint16_t> proj;     // [2 halves][ATILES][KSTEPS_P][64 lanes][8] bf16 bits
  std::vector<uint16_t> rebuild;  // [2 halves][QTILES][KSTEPS_R][64 lanes][8] bf16 bits
  std::vector<double> cons;       // MfmaConsLayout<N>
};

// Tables of a context: Q1-point 1D stencil e1 (ascending) with weights w1 and lattice constant r,
// Hermite order N.  False if the 5 x 5 correction matrix is singular.
bool build_mfma_tables(int Q1, int N, double r, const double* w1, const int* e1, MfmaHostTables& out);

}  // namespace lbsmrt
