// Site-permutation group and its real irreps (host, FP64).
#pragma once

#include <cstdint>
#include <vector>

namespace ftlm {

struct Irrep {
  int dim = 0;
  int indicator = 0;               // Frobenius-Schur indicator
  std::vector<double> rho;         // |G| x dim x dim, row-major
  std::vector<double> chars;       // per class (canonical class order)
};

struct Group {
  int N = 0;
  int order = 0;
  std::vector<int32_t> perms;      // order x N, lexicographically sorted
  std::vector<uint16_t> mul;       // order x order: index of g*h
  std::vector<uint16_t> inv;       // order
  std::vector<int32_t> elem_order; // order
  std::vector<int32_t> class_of;   // order -> canonical class index
  std::vector<std::vector<int32_t>> classes;
  // irreps (empty when |G| is above the irrep limit)
  std::vector<Irrep> irreps;
  bool irreps_computed = false;
  bool all_real = false;           // every irrep has indicator +1 (and a real form)
  double max_residual = 0.0;

  int idx_mul(int a, int b) const { return mul[(size_t)a * order + b]; }
};

// Closure (Dimino's algorithm), tables, classes; throws ftlm::Error.
Group build_group(int N, const int32_t* gens, int ngens);
// Irreps from a random symmetric element of the right regular algebra.
void compute_irreps(Group& G);
// Largest residual of homomorphism, orthogonality of rho and great orthogonality.
double verify_irreps(const Group& G, const std::vector<const Irrep*>& irs);

// Symmetric eigen-decomposition by cyclic Jacobi rotations; A (n x n,
// row-major) is overwritten; V receives the eigenvectors as columns;
// eigenvalues are returned ascending with V's columns reordered to match.
std::vector<double> jacobi_eigh(std::vector<double>& A, int n, std::vector<double>& V);

}  // namespace ftlm
