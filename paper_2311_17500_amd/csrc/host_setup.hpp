// Host-side (CPU, FP64) setup of the space-time isogeometric operators.
//
// Everything computed here is small (1D data, at most a few hundred entries
// per direction): knot spans, B-spline values/derivatives at Gauss points,
// Greville abscissae, the univariate Galerkin matrices, the SU coefficients
// tau_k, the generalized eigendecompositions of the fast-diagonalization
// preconditioner and the gather tables that drive the GPU mode products.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace stiga {

// One univariate direction (a spatial direction or time).
struct Dir1D {
  int p = 0;            // degree
  int n = 0;            // number of B-splines
  int nel = 0;          // number of non-empty elements
  int nq = 0;           // Gauss points per element (p + 1)
  int Q = 0;            // total Gauss points (nel * nq)
  int nder = 0;         // highest stored derivative
  std::vector<double> knots;   // physical knots (time scaled by T)
  std::vector<double> brk;     // breakpoints
  std::vector<double> xq, wq;  // Gauss points / weights, element-major
  std::vector<int> first;      // index of the first non-zero basis function at each point
  std::vector<std::vector<double>> B;  // B[k][q*(p+1)+j] = k-th derivative of basis first[q]+j at xq[q]
  std::vector<double> grev;    // Greville abscissae (parametric)
  std::vector<double> grev_x;  // the same mapped to the physical axis (equal to grev for the identity map)
};

// Separable geometry map x = F(eta) of one spatial direction (the spatial
// part of the map G = (F, T tau) of Section 2 with a diagonal Jacobian):
// kind 0 identity, 1 affine F = a + (b - a) eta, 2 exponential grading
// F = a + (b - a) (exp(k eta) - 1) / (exp(k) - 1).  Rewrites the direction's
// Gauss data to physical quantities: points F(eta_q), weights w_q F'(eta_q),
// first derivatives b'/F', second derivatives b''/F'^2 - F'' b'/F'^3, and
// the mapped Greville abscissae; knots, spans and element windows stay
// parametric.  False with a message for invalid parameters.
bool apply_map(Dir1D& D, int kind, const double* param, std::string& err);

// Sparse row table for y[i] = sum_w coef[i*W+w] * x[col[i*W+w]].
struct Gather {
  int n_out = 0, W = 0;
  std::vector<int> col;
  std::vector<double> coef;
  // when every row reads the contiguous columns [c0[i], c0[i] + W) and c0 is
  // non-decreasing, c0 holds the window starts (empty otherwise)
  std::vector<int> c0;
};

// Rewrite each row of G as a contiguous window of W columns inside [0, n_in)
// (zero coefficients for padding) and fill G.c0 if the windows are monotone.
void make_contiguous(Gather& G, int n_in);

bool build_dir(const double* knots01, int nk, int p, double scale, int nder, Dir1D& out, std::string& err);

// Dense n x n matrices on the full basis: [i*n + j].
std::vector<double> gram1d(const Dir1D& D, int dtest, int dtrial, const std::vector<double>* wq_weight);

// SU coefficients tau_k (k = 1..p_t) evaluated at the time Gauss points:
// returns tauq[(k-1)*Q + q].  Square full-basis system, column-equilibrated LU.
bool tau_at_quad(const Dir1D& T, std::vector<double>& tauq, std::vector<double>& coefs, std::string& err);

// Symmetric-definite generalized eigenproblem K u = lambda M u (dense, n x n):
// U (column j = eigenvector j, row-major U[i*n+j]) with U^T M U = I, ascending lambda.
// Symmetric eigenproblem (Householder tridiagonalization + implicit-shift QL):
// lam ascending, eigenvectors in the columns of the row-major Q.
bool sym_eig(const std::vector<double>& A, int n, std::vector<double>& Q, std::vector<double>& lam, std::string& err);
bool gen_eig_sym(const std::vector<double>& K, const std::vector<double>& M, int n,
                 std::vector<double>& U, std::vector<double>& lam, std::string& err);

// Fast-diagonalization data for the time pencil (Section 3.2), real block form.
struct TimeFD {
  int N = 0;                    // N_t
  std::vector<double> U;        // N x N, row-major, U^T M_t U = I
  std::vector<double> mu;       // N-1 entries: block (2m, 2m+1) has skew value mu[2m] (= -mu[2m+1] pairing)
  std::vector<int> kind;        // N-1 entries: 0 = first of a 2x2 pair, 1 = second, 2 = single (zero block)
  std::vector<double> l;        // N-1 arrow entries
  double sigma = 0.0;           // corner
};
bool time_fd(const std::vector<double>& Wt, const std::vector<double>& Mt, int N, TimeFD& out, std::string& err);

// Gather tables.
Gather banded_table(const std::vector<double>& A, int n, int row0, int nrow, int bw);
Gather eval_table(const Dir1D& D, int der);             // Q x n (expansion to Gauss points)
Gather eval_table_T(const Dir1D& D, int der, const std::vector<double>* wscale);  // n x Q (projection)
// Projection onto the streamline test functions b_i + tau b_i' (tau per Gauss
// point), same layout as eval_table_T(D, 0, nullptr).
Gather streamline_table_T(const Dir1D& D, const std::vector<double>& tau);
Gather dense_table(const std::vector<double>& A, int nrow, int ncol, bool transpose);

// Hat-function interpolation weights from nodes to points (constant extension outside).
void hat_weights(const std::vector<double>& nodes, const std::vector<double>& x,
                 std::vector<int>& left, std::vector<double>& wleft);

// B-spline values of all basis functions at arbitrary points (dense rows, n columns).
std::vector<double> collocation(const Dir1D& D, const std::vector<double>& x, int der);

// Element windows (support extensions) for full-basis indices [first, n): [e0, e1) per index.
void support_windows(const Dir1D& D, int first, std::vector<int>& e0, std::vector<int>& e1);

}  // namespace stiga
