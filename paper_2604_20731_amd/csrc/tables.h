// Host-side float64 tables of the discretisation (basis values, quadrature,
// 1D mass bands, projection weights, DST-I basis, well sources).  Built once
// per context at init; the device receives them converted to the working
// precision.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace crv {

// (r+1)-point Gauss-Legendre rule on [0,1]: points and weights.
void gauss_rule01(int npts, std::vector<double>& x, std::vector<double>& w);

// Values (and first derivatives) of the r+1 B-splines that are nonzero on the
// knot span containing x (open uniform knots, Ne elements, degree r).
// first = global index of the first of them.
void local_basis(int ne, int r, double x, double* val, double* der, int* first);

// Banded 1D mass matrix: band[i*(r+1) + t] = int B_i B_{i+t}, t = 0..r.
std::vector<double> mass_band(int ne, int r);

// Projection weights Q(k, i) = int B_k(x) hat_i(x) dx; the nonzeros of row k
// are nodes first(k) .. first(k)+r+1, stored qv[k*(r+2) + t].
void projection_table(int ne, int r, std::vector<int>& first, std::vector<double>& qv);

// Knot values: at node x_i = i/Ne, B-spline values of indices
// first(i)..first(i)+r, stored kv[i*(r+1) + t].
void knot_table(int ne, int r, std::vector<int>& first, std::vector<double>& kv);

// Per element e and Gauss point g (r+1 per element): values and derivatives
// of the r+1 local basis functions (global indices e..e+r), and the local
// coordinate xi in [0,1] of every Gauss point and its weight (times h_e).
void gauss_tables(int ne, int r, std::vector<double>& gb, std::vector<double>& gdb,
                  std::vector<double>& xi, std::vector<double>& w);

// Orthonormal DST-I basis of size m, padded to mp x mp with zeros:
// S(k, j) = sqrt(2/(m+1)) sin((k+1)(j+1) pi/(m+1)); lam[k] = 4 sin^2((k+1) pi/(2(m+1))).
void dst_table(int m, int mp, std::vector<double>& s, std::vector<double>& lam);
// Symbols of the uniform degree-r B-spline mass and stiffness (unit spacing)
// at the DST-I frequencies theta_k = (k+1) pi/(m+1), k < m:
//   m(theta) = M_0 + 2 sum_t M_t cos(t theta),  k(theta) likewise,
// with M_t = N_{2r+1}(r+1+t), K_t = -N''_{2r+1}(r+1+t) the autocorrelations of
// the cardinal B-spline N_r (support [0, r+1]) and of its derivative.
// sym = (m_0 .. m_{mp-1}, k_0 .. k_{mp-1}), padded modes 1.
void bspline_symbols(int r, int m, int mp, std::vector<double>& sym);
// A (M x K row-major, M multiple of 32, K of 16) rearranged into the packed
// operand order of the float32 32x32x2 matrix-core product: index
// ((mb * K/16 + kc) * 64 + lane) * 8 + u holds A[32 mb + lane%32][16 kc + 2u + lane/32].
std::vector<double> pack_gemm_a(const std::vector<double>& a, int M, int K);

// Well sources on the nodal grid (injectors and producers separate).
// Returns false with a message if a well covers no node or a boundary node.
bool well_sources(const double* wells, int n_wells, int ne, int dim, double radius,
                  std::vector<double>& q_inj, std::vector<double>& q_prod, std::string& err);

}  // namespace crv
