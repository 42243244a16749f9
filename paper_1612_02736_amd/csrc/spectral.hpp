// Spectral primitives on [-1, 1] for the planner (host, FP64).
//
// Paper Sec. 3.1-3.4: a p-point Chebyshev grid per direction including the
// end points (|I_ce| = 4(p-1)), q Gauss-Legendre nodes per side, spectral
// differentiation exact for degree <= p-1, and interpolation between the two
// families (corner values by extrapolation).
#pragma once
#include <vector>

namespace hps {

// Chebyshev-Lobatto points, ascending.
std::vector<double> cheb_points(int p);
// Roots of the Legendre polynomial P_q, ascending (Newton on the three-term
// recurrence from the asymptotic initial guesses).
std::vector<double> legendre_roots(int q);
// Barycentric weights of arbitrary distinct nodes.
std::vector<double> bary_weights(const std::vector<double> &x);
// Row-major n x n differentiation matrix D[i*n+j] = l_j'(x_i) (barycentric
// off-diagonal entries, diagonal by the zero-row-sum identity).
std::vector<double> diff_matrix(const std::vector<double> &x);
// Row-major (dst.size() x src.size()) interpolation matrix, second
// barycentric form; points outside the node range extrapolate.
std::vector<double> interp_matrix(const std::vector<double> &src,
                                  const std::vector<double> &dst);

}  // namespace hps
