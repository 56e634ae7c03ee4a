// host_setup.hpp -- host-side discretisation and solver setup of the pmgrit library.
//
// Everything here runs once per handle (pmgrit_create): it turns the paper's problem statement
// (degree p, mesh width h = 1/n, kappa, dt per time level) into the arrays the GPU kernels
// stream.  Structure exploited on the single-patch geometries the library supports: the
// parametrisations are separable (F(s,t) = (s,t) on the square; r(s) * c(t) on the quarter
// annulus), so with a tensor Gauss rule every 2D matrix is a short sum of Kronecker products of
// 1D weighted B-spline matrices.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace pmg {

// compressed sparse rows, sorted columns, FP64 values
struct Csr {
  int nr = 0, nc = 0;
  std::vector<int> rp, ci;
  std::vector<double> v;
  int nnz() const { return (int)ci.size(); }
};

// dense row-major matrix
struct Dense {
  int r = 0, c = 0;
  std::vector<double> a;
  Dense() = default;
  Dense(int r_, int c_) : r(r_), c(c_), a((size_t)r_ * c_, 0.0) {}
  double& operator()(int i, int j) { return a[(size_t)i * c + j]; }
  double operator()(int i, int j) const { return a[(size_t)i * c + j]; }
};

// Gauss-Legendre rule on [0,1] by the Golub-Welsch eigenvalue method
void gauss01(int q, std::vector<double>& x, std::vector<double>& w);

// symmetric eigen-decomposition by cyclic Jacobi rotations: A = Z diag(lam) Z^T
void sym_eig(const Dense& A, std::vector<double>& lam, Dense& Z);

// the p+1 non-zero B-splines of degree p (and first derivatives) at x in knot span `span`
void bspline_values(const std::vector<double>& knots, int p, int span, double x, double* val, double* der);

// 1D weighted matrices between degree pa (rows) and degree pb (cols) on n uniform elements:
// W_ij = int d^da phi_i * d^db phi_j * w(s) ds over [0,1], q Gauss points per element.
// Weight kinds: 0 -> 1, 1 -> r(s) = 1 + s, 2 -> 1 / r(s), 3 -> |c'(s)|, 4 -> 1 / |c'(s)| with c the
// rational quadratic quarter circle.  Full (boundary functions included) matrices.
Dense weighted_1d(int n, int pa, int pb, int da, int db, int wkind, int q);

// load vector of one 1D mode m(k, s) (k = 0 -> 1, else sin(k pi s)) against degree-p functions
std::vector<double> mode_load_1d(int n, int p, int k, int wkind, int q);

struct KronTerm {
  const Dense* Y;  // slow (second parameter direction) factor
  const Dense* X;  // fast (first direction) factor
  double c;
};

// CSR of sum_t c_t (Y_t kron X_t) restricted to the interior functions (first and last per
// direction dropped), pattern = tensor-product support overlap (|i - j| within the band)
Csr kron_interior(int Ny, int Nx, int My, int Mx, int bandy_lo, int bandy_hi, int bandx_lo, int bandx_hi,
                  const std::vector<KronTerm>& terms);

// ILUT with drop tolerance tau (relative to the row 2-norm) and per-row caps on the strict
// lower / strict upper parts; L strict lower (unit diagonal implied), U upper with the diagonal
// first in each row.  Returns false on a non-positive or non-finite pivot.
bool ilut(const Csr& A, double tau, const std::vector<int>& lcap, const std::vector<int>& ucap, Csr& L, Csr& U,
          std::string& err);

// Level schedule of a blocked triangular solve T y = r (T = L unit lower, or U upper).  Rows are
// cut into blocks of `bs` consecutive rows; every block's diagonal part is inverted densely, the
// rest (off-block entries) is applied as sparse rows; blocks are level-scheduled by their
// off-block dependencies.  Arrays are in "level order" (the rows of level 0, then level 1, ...;
// inside a level the rows of one block are consecutive).
struct TriSchedule {
  int n = 0, nlev = 0, nblocks = 0, bs = 1, max_rows = 0;
  bool upper = false;
  std::vector<int> lev_ptr;        // [nlev + 1] positions in the level-ordered row list
  std::vector<int> row;            // [n] row index of position q
  std::vector<int> orp, oci;       // off-block CSR in level order: orp[q]..orp[q+1]
  std::vector<double> ov;
  std::vector<int> dq0, dcnt;      // dense phase: s positions dq0[q] .. dq0[q]+dcnt[q]-1 (within level)
  std::vector<int64_t> doff;       //              values dval[doff[q] ..]
  std::vector<double> dval;
};
TriSchedule build_schedule(const Csr& T, bool upper, int bs, int cap);

// Exact p = 1 solve by fast diagonalisation: (G kron ...) see host_setup.cpp.
struct CoarseFdm {
  int n1 = 0;                      // interior functions per direction at p = 1
  std::vector<double> V;           // [n1 * n1] V[iy * n1 + k], generalized eigenvectors (second direction)
  std::vector<double> lam;         // [n1]
  std::vector<double> tl, tdinv;   // per level: [n1 modes * n1] Thomas multipliers and inverse pivots
};

}  // namespace pmg
