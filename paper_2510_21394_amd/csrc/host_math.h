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

// Even/odd splitting of the symmetric Toeplitz D = -h^{-alpha} Toeplitz(g).  D is
// persymmetric (J D J = D, J the exchange matrix), so with m = floor(n/2) the orthogonal
// Z whose columns are (e_k + e_{n-1-k})/sqrt(2) (k < m), e_m (odd n only), then
// (e_k - e_{n-1-k})/sqrt(2) (k < m) block-diagonalises it: Z^T D Z = diag(De, Do), De of
// size me = n - m, Do of size mo = m, with (i, k < m, t_k = D[0][k])
//   De[i][k] = t_|i-k| + t_{n-1-i-k},  Do[i][k] = t_|i-k| - t_{n-1-i-k},
//   De[i][m] = De[m][i] = sqrt(2) t_{m-i},  De[m][m] = t_0   (odd n).
// Each block is diagonalised by sym_eig, then given one Newton-Schulz orthogonalisation
// sweep and Rayleigh-quotient eigenvalues in long double; Q = Z diag(Ve, Vo) is rounded once
// from long double with its mirror entries copied, so Q[n-1-i][k] = +-Q[i][k] holds exactly
// (+ for the me even columns, - for the mo odd ones).
struct SplitEig {
  int64_t n = 0, me = 0, mo = 0;
  std::vector<double> Q;    // n x n row-major, column k <-> lam[k]
  std::vector<double> lam;  // block order: even block (ascending), then odd block (ascending)
};
bool toeplitz_eig_split(int64_t n, double alpha, double h, int fd_order, SplitEig& s);

// The stacked even/odd block matrices of the split mode products, read off Q (n x n,
// exact even/odd structure, block order), each block ld x ld zero padded (ld >= me):
//   F = [Fe; Fo] (forward, Q^T):  Fe[i][k] = Q[k][i] (k < m), Q[m][i]/2 (k = m, odd n);
//                                 Fo[i][k] = Q[k][me + i]
//   B = [Be; Bo] (backward, Q):   Be[i][k] = Q[i][k];  Bo[i][k] = Q[i][me + k]
// so that the split products are the dense ones with the same Q, summed in another order.
void split_block_matrices(int64_t n, int64_t me, int64_t mo, const std::vector<double>& Q, int64_t ld,
                          std::vector<double>& F, std::vector<double>& B);

// Round a double to the nearest bfloat16 (ties to even); returns the bf16 bits.
uint16_t bf16_round(double x);
double bf16_value(uint16_t b);

}  // namespace fcgle
