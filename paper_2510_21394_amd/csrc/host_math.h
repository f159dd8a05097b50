// Host-side FP64 numerics of the plan set-up: FD weights, the dense Toeplitz
// matrix, its symmetric eigendecomposition, scalar matrix functions and the
// BF16 splitting of Q.  No HIP calls.
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

namespace fcgle {

// g_0..g_{n-1}: order 2 by the recurrence of Section 2, order 4 by eq. FD4.
std::vector<double> fd_weights(double alpha, int64_t n, int fd_order);

// Eigendecomposition of a symmetric n x n row-major matrix A (destroyed).
// On return lambda is ascending and Q (row-major) has the eigenvector of
// lambda[k] in column k.  Returns false if the QR sweep did not converge.
bool sym_eig(int64_t n, std::vector<double>& A, std::vector<double>& Q, std::vector<double>& lambda);

// D = -h^{-alpha} Toeplitz(g) followed by sym_eig.
bool toeplitz_eig(int64_t n, double alpha, double h, int fd_order, std::vector<double>& Q,
                  std::vector<double>& lambda);

// Round a double to the nearest bfloat16 (ties to even); returns the bf16 bits.
uint16_t bf16_round(double x);
double bf16_value(uint16_t b);

}  // namespace fcgle
