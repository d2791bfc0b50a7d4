// Host-side FP64 setup: univariate B-splines (Section 2), Galerkin matrices
// (Section 3.1.1), SU coefficients tau_k (eq. (3.5)), fast-diagonalization
// factors (Section 3.2) and the gather tables of the GPU mode products.
#include "host_setup.hpp"

#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>

namespace stiga {
namespace {

// Index i of the knot span with knots[i] <= x < knots[i+1], limited to the
// non-degenerate range [p, n-1]; the right end maps to the last non-empty span.
int find_span(const std::vector<double>& kn, int p, double x) {
  const int n = static_cast<int>(kn.size()) - p - 1;
  if (x >= kn[n]) {
    int i = n - 1;
    while (i > p && kn[i] == kn[i + 1]) --i;
    return i;
  }
  int i = static_cast<int>(std::upper_bound(kn.begin(), kn.end(), x) - kn.begin()) - 1;
  return std::min(std::max(i, p), n - 1);
}

// k-th derivative of the degree-q B-spline j at x, from the table of values of
// all non-zero lower-degree functions on span `span`:
//   d^k b_{j,q} = q ( d^{k-1} b_{j,q-1} / (xi_{j+q} - xi_j)
//                   - d^{k-1} b_{j+1,q-1} / (xi_{j+q+1} - xi_{j+1}) ).
double dval(const std::vector<double>& kn, const std::vector<std::vector<double>>& N, int span, int k,
            int q, int j) {
  if (k > q) return 0.0;
  if (k == 0) {
    const int r = j - (span - q);
    return (r >= 0 && r <= q) ? N[q][r] : 0.0;
  }
  double out = 0.0;
  const double d1 = kn[j + q] - kn[j];
  const double d2 = kn[j + q + 1] - kn[j + 1];
  if (d1 != 0.0) out += dval(kn, N, span, k - 1, q - 1, j) / d1;
  if (d2 != 0.0) out -= dval(kn, N, span, k - 1, q - 1, j + 1) / d2;
  return q * out;
}

// Values (and derivatives up to nd) of the p+1 functions b_{span-p..span} at x.
// out[k*(p+1) + r] = d^k b_{span-p+r}(x).
void basis_ders(const std::vector<double>& kn, int p, int span, double x, int nd, double* out) {
  std::vector<std::vector<double>> N(p + 1);
  N[0] = {1.0};
  for (int q = 1; q <= p; ++q) {
    N[q].assign(q + 1, 0.0);
    for (int r = 0; r <= q; ++r) {
      const int j = span - q + r;
      double v = 0.0;
      if (r >= 1) {  // b_{j,q-1} is non-zero on this span
        const double den = kn[j + q] - kn[j];
        if (den != 0.0) v += (x - kn[j]) / den * N[q - 1][r - 1];
      }
      if (r <= q - 1) {  // b_{j+1,q-1}
        const double den = kn[j + q + 1] - kn[j + 1];
        if (den != 0.0) v += (kn[j + q + 1] - x) / den * N[q - 1][r];
      }
      N[q][r] = v;
    }
  }
  for (int k = 0; k <= nd; ++k)
    for (int r = 0; r <= p; ++r) out[k * (p + 1) + r] = dval(kn, N, span, k, p, span - p + r);
}

// Gauss-Legendre rule on [0, 1] by Newton's method on P_n.
void gauss01(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    // recompute derivative at the converged root
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = (n == 1) ? 1.0 : n * (z * p1 - p0) / (z * z - 1.0);
    x[n - 1 - i] = 0.5 * (z + 1.0);
    w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);
  }
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return x[a] < x[b]; });
  std::vector<double> xs(n), ws(n);
  for (int i = 0; i < n; ++i) { xs[i] = x[idx[i]]; ws[i] = w[idx[i]]; }
  x = xs;
  w = ws;
}

// Dense LU with partial pivoting (row-major n x n), in place; returns false if singular.
bool lu_factor(std::vector<double>& A, int n, std::vector<int>& piv) {
  piv.resize(n);
  for (int c = 0; c < n; ++c) {
    int pr = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[pr * n + c])) pr = r;
    piv[c] = pr;
    if (A[pr * n + c] == 0.0) return false;
    if (pr != c)
      for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[pr * n + k]);
    for (int r = c + 1; r < n; ++r) {
      const double f = A[r * n + c] / A[c * n + c];
      A[r * n + c] = f;
      for (int k = c + 1; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
    }
  }
  return true;
}

void lu_solve(const std::vector<double>& LU, int n, const std::vector<int>& piv, std::vector<double>& b) {
  for (int c = 0; c < n; ++c) std::swap(b[c], b[piv[c]]);
  for (int r = 1; r < n; ++r)
    for (int k = 0; k < r; ++k) b[r] -= LU[r * n + k] * b[k];
  for (int r = n - 1; r >= 0; --r) {
    for (int k = r + 1; k < n; ++k) b[r] -= LU[r * n + k] * b[k];
    b[r] /= LU[r * n + r];
  }
}

bool cholesky(const std::vector<double>& M, int n, std::vector<double>& L) {
  L.assign(static_cast<size_t>(n) * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = M[j * n + j];
    for (int k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
    if (!(s > 0.0)) return false;
    L[j * n + j] = std::sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = M[i * n + j];
      for (int k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = t / L[j * n + j];
    }
  }
  return true;
}

// X = L^{-1} A (A is n x m, row-major), forward substitution column by column.
void lower_solve(const std::vector<double>& L, int n, std::vector<double>& A, int m) {
  for (int c = 0; c < m; ++c)
    for (int i = 0; i < n; ++i) {
      double s = A[i * m + c];
      for (int k = 0; k < i; ++k) s -= L[i * n + k] * A[k * m + c];
      A[i * m + c] = s / L[i * n + i];
    }
}

// X = L^{-T} A.
void upper_solve_T(const std::vector<double>& L, int n, std::vector<double>& A, int m) {
  for (int c = 0; c < m; ++c)
    for (int i = n - 1; i >= 0; --i) {
      double s = A[i * m + c];
      for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * A[k * m + c];
      A[i * m + c] = s / L[i * n + i];
    }
}

}  // namespace

bool build_dir(const double* knots01, int nk, int p, double scale, int nder, Dir1D& D, std::string& err) {
  if (p < 1) { err = "degree must be >= 1"; return false; }
  if (nk < 2 * (p + 1)) { err = "knot vector too short"; return false; }
  for (int i = 0; i + 1 < nk; ++i)
    if (!(knots01[i] <= knots01[i + 1])) { err = "knots must be non-decreasing"; return false; }
  for (int i = 0; i <= p; ++i)
    if (knots01[i] != 0.0 || knots01[nk - 1 - i] != 1.0) { err = "knot vector must be open on [0,1]"; return false; }
  // interior multiplicity <= p (C^0 at least)
  for (int i = p + 1; i < nk - p - 1;) {
    int j = i;
    while (j < nk - p - 1 && knots01[j] == knots01[i]) ++j;
    if (j - i > p) { err = "interior knot multiplicity exceeds the degree"; return false; }
    i = j;
  }
  D.p = p;
  D.knots.resize(nk);
  for (int i = 0; i < nk; ++i) D.knots[i] = scale * knots01[i];
  D.n = nk - p - 1;
  D.brk.clear();
  for (double v : D.knots)
    if (D.brk.empty() || v != D.brk.back()) D.brk.push_back(v);
  D.nel = static_cast<int>(D.brk.size()) - 1;
  D.nq = p + 1;
  D.Q = D.nel * D.nq;
  D.nder = nder;
  std::vector<double> g, gw;
  gauss01(D.nq, g, gw);
  D.xq.resize(D.Q);
  D.wq.resize(D.Q);
  D.first.resize(D.Q);
  D.B.assign(nder + 1, std::vector<double>(static_cast<size_t>(D.Q) * (p + 1)));
  std::vector<double> tmp((nder + 1) * (p + 1));
  for (int e = 0; e < D.nel; ++e) {
    const double a = D.brk[e], h = D.brk[e + 1] - D.brk[e];
    for (int k = 0; k < D.nq; ++k) {
      const int q = e * D.nq + k;
      const double x = a + h * g[k];
      D.xq[q] = x;
      D.wq[q] = h * gw[k];
      const int span = find_span(D.knots, p, x);
      D.first[q] = span - p;
      basis_ders(D.knots, p, span, x, nder, tmp.data());
      for (int dk = 0; dk <= nder; ++dk)
        for (int r = 0; r <= p; ++r) D.B[dk][static_cast<size_t>(q) * (p + 1) + r] = tmp[dk * (p + 1) + r];
    }
  }
  D.grev.resize(D.n);
  for (int i = 0; i < D.n; ++i) {
    double s = 0.0;
    for (int k = i + 1; k <= i + p; ++k) s += D.knots[k];
    D.grev[i] = s / p;
  }
  D.grev_x = D.grev;
  return true;
}

bool apply_map(Dir1D& D, int kind, const double* prm, std::string& err) {
  if (kind == 0) return true;
  if (kind != 1 && kind != 2) { err = "unknown geometry map"; return false; }
  const double a = prm[0], b = prm[1], k = prm[2];
  if (!(b > a) || !std::isfinite(a) || !std::isfinite(b)) { err = "geometry map needs a < b"; return false; }
  if (kind == 2 && (!(std::fabs(k) > 1e-8) || !(std::fabs(k) < 50.0))) {
    err = "graded geometry map needs 1e-8 < |k| < 50";
    return false;
  }
  // F, F', F'' at a parametric point
  auto map = [&](double e, double& F, double& F1, double& F2) {
    if (kind == 1) {
      F = a + (b - a) * e;
      F1 = b - a;
      F2 = 0.0;
    } else {
      const double den = std::expm1(k);
      F = a + (b - a) * std::expm1(k * e) / den;
      F1 = (b - a) * k * std::exp(k * e) / den;
      F2 = k * F1;
    }
  };
  const int p1 = D.p + 1;
  for (int q = 0; q < D.Q; ++q) {
    double F, F1, F2;
    map(D.xq[q], F, F1, F2);
    D.xq[q] = F;
    D.wq[q] *= F1;
    for (int r = 0; r < p1; ++r) {
      const size_t i = static_cast<size_t>(q) * p1 + r;
      const double d1 = D.B[1][i];
      if (D.nder >= 2) D.B[2][i] = D.B[2][i] / (F1 * F1) - F2 * d1 / (F1 * F1 * F1);
      D.B[1][i] = d1 / F1;
    }
  }
  for (int i = 0; i < D.n; ++i) {
    double F, F1, F2;
    map(D.grev[i], F, F1, F2);
    D.grev_x[i] = F;
  }
  return true;
}

std::vector<double> gram1d(const Dir1D& D, int dt, int dj, const std::vector<double>* wt) {
  const int n = D.n, p = D.p;
  std::vector<double> G(static_cast<size_t>(n) * n, 0.0);
  for (int q = 0; q < D.Q; ++q) {
    const double w = D.wq[q] * (wt ? (*wt)[q] : 1.0);
    const int f = D.first[q];
    for (int a = 0; a <= p; ++a)
      for (int b = 0; b <= p; ++b)
        G[static_cast<size_t>(f + a) * n + (f + b)] +=
            w * D.B[dt][static_cast<size_t>(q) * (p + 1) + a] * D.B[dj][static_cast<size_t>(q) * (p + 1) + b];
  }
  return G;
}

std::vector<double> collocation(const Dir1D& D, const std::vector<double>& x, int der) {
  const int n = D.n, p = D.p;
  std::vector<double> C(x.size() * static_cast<size_t>(n), 0.0);
  std::vector<double> tmp((der + 1) * (p + 1));
  for (size_t m = 0; m < x.size(); ++m) {
    const int span = find_span(D.knots, p, x[m]);
    basis_ders(D.knots, p, span, x[m], der, tmp.data());
    for (int r = 0; r <= p; ++r) C[m * n + span - p + r] = tmp[der * (p + 1) + r];
  }
  return C;
}

bool tau_at_quad(const Dir1D& T, std::vector<double>& tauq, std::vector<double>& coefs, std::string& err) {
  const int p = T.p, nt = T.n;
  // full-basis time-derivative matrix W[i][j] = int b_j' b_i
  std::vector<double> W = gram1d(T, 0, 1, nullptr);
  // spaces of tau_k: degree p-k, maximal regularity on the breakpoints
  struct Space { int q; std::vector<double> kn; int n; std::vector<double> val; };  // val[Q][n] dense
  std::vector<Space> sp(p);
  int ncols = 0;
  for (int k = 1; k <= p; ++k) {
    Space& s = sp[k - 1];
    s.q = p - k;
    s.kn.assign(s.q + 1, T.brk.front());
    for (size_t i = 1; i + 1 < T.brk.size(); ++i) s.kn.push_back(T.brk[i]);
    for (int i = 0; i <= s.q; ++i) s.kn.push_back(T.brk.back());
    s.n = static_cast<int>(s.kn.size()) - s.q - 1;
    s.val.assign(static_cast<size_t>(T.Q) * s.n, 0.0);
    std::vector<double> tmp(s.q + 1);
    for (int qq = 0; qq < T.Q; ++qq) {
      const int span = find_span(s.kn, s.q, T.xq[qq]);
      basis_ders(s.kn, s.q, span, T.xq[qq], 0, tmp.data());
      for (int r = 0; r <= s.q; ++r) s.val[static_cast<size_t>(qq) * s.n + span - s.q + r] = tmp[r];
    }
    ncols += s.n;
  }
  std::vector<std::pair<int, int>> rows;
  for (int i = 0; i + 1 < nt; ++i)
    for (int l = 1; l <= std::min(p, nt - 1 - i); ++l) rows.emplace_back(i, l);
  const int nr = static_cast<int>(rows.size());
  if (nr != ncols) { err = "tau system is not square"; return false; }
  std::vector<double> A(static_cast<size_t>(nr) * nr, 0.0), rhs(nr);
  for (int r = 0; r < nr; ++r) {
    const int i = rows[r].first, j = rows[r].first + rows[r].second;
    rhs[r] = -W[static_cast<size_t>(i) * nt + j];
    int c0 = 0;
    for (int k = 1; k <= p; ++k) {
      const Space& s = sp[k - 1];
      for (int qq = 0; qq < T.Q; ++qq) {
        const int f = T.first[qq];
        if (i < f || j > f + p) continue;  // both functions must be non-zero at the point
        const double prod = T.wq[qq] * T.B[k][static_cast<size_t>(qq) * (p + 1) + (i - f)] *
                            T.B[k][static_cast<size_t>(qq) * (p + 1) + (j - f)];
        for (int c = 0; c < s.n; ++c) A[static_cast<size_t>(r) * nr + c0 + c] += prod * s.val[static_cast<size_t>(qq) * s.n + c];
      }
      c0 += s.n;
    }
  }
  // column equilibration, LU with partial pivoting, two refinement steps in long double
  std::vector<double> scale(nr, 0.0);
  for (int c = 0; c < nr; ++c) {
    for (int r = 0; r < nr; ++r) scale[c] = std::max(scale[c], std::fabs(A[static_cast<size_t>(r) * nr + c]));
    if (scale[c] == 0.0) scale[c] = 1.0;
  }
  std::vector<double> As(A);
  for (int r = 0; r < nr; ++r)
    for (int c = 0; c < nr; ++c) As[static_cast<size_t>(r) * nr + c] /= scale[c];
  std::vector<double> LU(As);
  std::vector<int> piv;
  if (!lu_factor(LU, nr, piv)) { err = "tau system is singular"; return false; }
  std::vector<double> y(rhs);
  lu_solve(LU, nr, piv, y);
  for (int it = 0; it < 2; ++it) {
    std::vector<double> res(nr);
    for (int r = 0; r < nr; ++r) {
      long double s = rhs[r];
      for (int c = 0; c < nr; ++c) s -= static_cast<long double>(As[static_cast<size_t>(r) * nr + c]) * y[c];
      res[r] = static_cast<double>(s);
    }
    lu_solve(LU, nr, piv, res);
    for (int c = 0; c < nr; ++c) y[c] += res[c];
  }
  coefs.resize(nr);
  for (int c = 0; c < nr; ++c) coefs[c] = y[c] / scale[c];
  tauq.assign(static_cast<size_t>(p) * T.Q, 0.0);
  int c0 = 0;
  for (int k = 1; k <= p; ++k) {
    const Space& s = sp[k - 1];
    for (int qq = 0; qq < T.Q; ++qq) {
      double v = 0.0;
      for (int c = 0; c < s.n; ++c) v += s.val[static_cast<size_t>(qq) * s.n + c] * coefs[c0 + c];
      tauq[static_cast<size_t>(k - 1) * T.Q + qq] = v;
    }
    c0 += s.n;
  }
  return true;
}

// Symmetric eigenproblem A = Q diag(lam) Q^T (Golub and Van Loan, "Matrix
// Computations", Sections 8.3.1-8.3.3): an orthogonal similarity to
// tridiagonal form by Householder reflections, then implicit QR steps with
// the Wilkinson shift on the tridiagonal matrix, each step chasing the bulge
// down with Givens rotations; every transformation is accumulated into Q.
// Off-diagonal entries below eps_mach (|t_ii| + |t_jj|) are set to zero
// (deflation).  Output as gen_eig_sym: lam ascending, eigenvectors in the
// columns of the row-major Q.  O(n^3), unlike the cyclic Jacobi sweeps.
bool sym_eig(const std::vector<double>& A, int n, std::vector<double>& Q, std::vector<double>& lam, std::string& err) {
  for (double v : A)
    if (!std::isfinite(v)) {
      err = "non-finite matrix entry";
      return false;
    }
  auto at = [n](std::vector<double>& M, int i, int j) -> double& { return M[static_cast<size_t>(i) * n + j]; };
  std::vector<double> T(A);                               // working copy, reduced in place
  std::vector<double> V(static_cast<size_t>(n) * n, 0.0);  // accumulated transformations
  for (int i = 0; i < n; ++i) at(V, i, i) = 1.0;
  // ---- phase 1: T <- H T H column by column, H = I - beta v v^T zeroing T[k+2:, k]
  std::vector<double> v(n), pv(n), wv(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;   // length of the column part x = T[k+1:, k]
    double xn2 = 0.0;
    for (int i = 1; i < m; ++i) xn2 += at(T, k + 1 + i, k) * at(T, k + 1 + i, k);
    if (xn2 == 0.0) continue;   // already tridiagonal in this column
    const double x0 = at(T, k + 1, k);
    const double alpha = -std::copysign(std::sqrt(x0 * x0 + xn2), x0);   // H x = alpha e_1
    // v = x - alpha e_1, beta = 2 / (v^T v)
    v[0] = x0 - alpha;
    for (int i = 1; i < m; ++i) v[i] = at(T, k + 1 + i, k);
    const double vtv = v[0] * v[0] + xn2;
    const double beta = 2.0 / vtv;
    // trailing block B = T[k+1:, k+1:]:  p = beta B v,  w = p - (beta p^T v / 2) v,
    // B <- B - v w^T - w v^T
    double pv_dot = 0.0;
    for (int i = 0; i < m; ++i) {
      double acc = 0.0;
      for (int j = 0; j < m; ++j) acc += at(T, k + 1 + i, k + 1 + j) * v[j];
      pv[i] = beta * acc;
      pv_dot += pv[i] * v[i];
    }
    const double half = 0.5 * beta * pv_dot;
    for (int i = 0; i < m; ++i) wv[i] = pv[i] - half * v[i];
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) at(T, k + 1 + i, k + 1 + j) -= v[i] * wv[j] + wv[i] * v[j];
    at(T, k + 1, k) = at(T, k, k + 1) = alpha;
    for (int i = 1; i < m; ++i) at(T, k + 1 + i, k) = at(T, k, k + 1 + i) = 0.0;
    // V <- V H (columns k+1..n-1)
    for (int r = 0; r < n; ++r) {
      double acc = 0.0;
      for (int j = 0; j < m; ++j) acc += at(V, r, k + 1 + j) * v[j];
      acc *= beta;
      for (int j = 0; j < m; ++j) at(V, r, k + 1 + j) -= acc * v[j];
    }
  }
  std::vector<double> dg(n), od(std::max(n - 1, 1), 0.0);   // diagonal, off-diagonal (od[i] = t_{i,i+1})
  for (int i = 0; i < n; ++i) dg[i] = at(T, i, i);
  for (int i = 0; i + 1 < n; ++i) od[i] = at(T, i + 1, i);
  // ---- phase 2: implicit Wilkinson-shift QR on the unreduced trailing blocks
  const double eps = std::numeric_limits<double>::epsilon();
  auto negligible = [&](int i) { return std::fabs(od[i]) <= eps * (std::fabs(dg[i]) + std::fabs(dg[i + 1])); };
  int hi = n - 1;
  long steps = 0;
  const long max_steps = 40L * std::max(n, 1);
  while (hi > 0) {
    if (negligible(hi - 1)) {
      od[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && !negligible(lo - 1)) --lo;
    if (++steps > max_steps) {
      err = "symmetric QR iteration did not converge";
      return false;
    }
    // Wilkinson shift: the eigenvalue of the trailing 2x2 block closer to t_hh
    const double h = 0.5 * (dg[hi - 1] - dg[hi]);
    const double e2 = od[hi - 1] * od[hi - 1];
    const double mu = dg[hi] - e2 / (h + (h >= 0.0 ? 1.0 : -1.0) * std::sqrt(h * h + e2));
    // rotation k acts on rows/columns (k, k+1) of the block; its first column
    // is proportional to (t_ll - mu, t_{l+1,l}), the later ones remove the bulge
    double x = dg[lo] - mu, z = od[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = std::hypot(x, z);
      const double cs = r > 0.0 ? x / r : 1.0;
      const double sn = r > 0.0 ? -z / r : 0.0;
      if (k > lo) od[k - 1] = r;
      const double a0 = dg[k], a1 = dg[k + 1], b0 = od[k];
      dg[k] = cs * cs * a0 - 2.0 * cs * sn * b0 + sn * sn * a1;
      dg[k + 1] = sn * sn * a0 + 2.0 * cs * sn * b0 + cs * cs * a1;
      od[k] = cs * sn * (a0 - a1) + (cs * cs - sn * sn) * b0;
      if (k + 1 < hi) {
        z = -sn * od[k + 1];   // bulge at (k, k+2)
        od[k + 1] *= cs;
        x = od[k];
      }
      for (int r2 = 0; r2 < n; ++r2) {
        const double qa = at(V, r2, k), qb = at(V, r2, k + 1);
        at(V, r2, k) = cs * qa - sn * qb;
        at(V, r2, k + 1) = sn * qa + cs * qb;
      }
    }
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int x, int y) { return dg[x] < dg[y]; });
  Q.assign(static_cast<size_t>(n) * n, 0.0);
  lam.resize(n);
  for (int j = 0; j < n; ++j) {
    lam[j] = dg[order[j]];
    for (int i = 0; i < n; ++i) Q[static_cast<size_t>(i) * n + j] = at(V, i, order[j]);
  }
  return true;
}

bool gen_eig_sym(const std::vector<double>& K, const std::vector<double>& M, int n, std::vector<double>& U,
                 std::vector<double>& lam, std::string& err) {
  std::vector<double> L;
  if (!cholesky(M, n, L)) { err = "mass matrix is not positive definite"; return false; }
  std::vector<double> C(K);
  lower_solve(L, n, C, n);                       // L^{-1} K
  std::vector<double> Ct(static_cast<size_t>(n) * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Ct[static_cast<size_t>(i) * n + j] = C[static_cast<size_t>(j) * n + i];
  lower_solve(L, n, Ct, n);                      // L^{-1} (L^{-1} K)^T = L^{-1} K L^{-T}
  for (int i = 0; i < n; ++i)                    // symmetrize
    for (int j = i + 1; j < n; ++j) {
      const double v = 0.5 * (Ct[static_cast<size_t>(i) * n + j] + Ct[static_cast<size_t>(j) * n + i]);
      Ct[static_cast<size_t>(i) * n + j] = Ct[static_cast<size_t>(j) * n + i] = v;
    }
  std::vector<double> Q, l;
  if (!sym_eig(Ct, n, Q, l, err)) return false;
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return l[a] < l[b]; });
  std::vector<double> Qs(static_cast<size_t>(n) * n);
  lam.resize(n);
  for (int j = 0; j < n; ++j) {
    lam[j] = l[idx[j]];
    for (int i = 0; i < n; ++i) Qs[static_cast<size_t>(i) * n + j] = Q[static_cast<size_t>(i) * n + idx[j]];
  }
  upper_solve_T(L, n, Qs, n);                    // U = L^{-T} Q
  U = Qs;
  return true;
}

bool time_fd(const std::vector<double>& Wt, const std::vector<double>& Mt, int N, TimeFD& F, std::string& err) {
  F.N = N;
  const int n = N - 1;
  if (n < 1) { err = "need at least two time unknowns"; return false; }
  std::vector<double> Wo(static_cast<size_t>(n) * n), Mo(static_cast<size_t>(n) * n), w(n), m(n);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) {
      Wo[static_cast<size_t>(i) * n + j] = Wt[static_cast<size_t>(i) * N + j];
      Mo[static_cast<size_t>(i) * n + j] = Mt[static_cast<size_t>(i) * N + j];
    }
    w[i] = Wt[static_cast<size_t>(i) * N + N - 1];
    m[i] = Mt[static_cast<size_t>(i) * N + N - 1];
  }
  std::vector<double> L;
  if (!cholesky(Mo, n, L)) { err = "time mass matrix is not positive definite"; return false; }
  // C = L^{-1} Wo L^{-T}, skew-symmetric
  std::vector<double> C(Wo);
  lower_solve(L, n, C, n);
  std::vector<double> Ct(static_cast<size_t>(n) * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Ct[static_cast<size_t>(i) * n + j] = C[static_cast<size_t>(j) * n + i];
  lower_solve(L, n, Ct, n);
  // Ct now holds L^{-1} Wo^T L^{-T} = -C for skew Wo; store C, exactly skew
  for (int i = 0; i < n; ++i) {
    Ct[static_cast<size_t>(i) * n + i] = 0.0;
    for (int j = i + 1; j < n; ++j) {
      const double v = -0.5 * (Ct[static_cast<size_t>(i) * n + j] - Ct[static_cast<size_t>(j) * n + i]);
      Ct[static_cast<size_t>(i) * n + j] = v;
      Ct[static_cast<size_t>(j) * n + i] = -v;
    }
  }
  // S = C^T C (symmetric PSD) has eigenvalues mu^2 in pairs
  std::vector<double> S(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += Ct[static_cast<size_t>(k) * n + i] * Ct[static_cast<size_t>(k) * n + j];
      S[static_cast<size_t>(i) * n + j] = s;
    }
  std::vector<double> V, mu2;
  if (!sym_eig(S, n, V, mu2, err)) return false;
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return mu2[a] > mu2[b]; });
  const double top = std::max(mu2[idx[0]], 1e-300);
  std::vector<double> Q(static_cast<size_t>(n) * n, 0.0);
  F.kind.assign(n, 2);
  int col = 0;
  auto put = [&](std::vector<double>& v) {  // Gram-Schmidt against previous columns, then store
    for (int pass = 0; pass < 2; ++pass)
      for (int c = 0; c < col; ++c) {
        double d = 0.0;
        for (int i = 0; i < n; ++i) d += Q[static_cast<size_t>(i) * n + c] * v[i];
        for (int i = 0; i < n; ++i) v[i] -= d * Q[static_cast<size_t>(i) * n + c];
      }
    double nr = 0.0;
    for (double x : v) nr += x * x;
    nr = std::sqrt(nr);
    for (int i = 0; i < n; ++i) Q[static_cast<size_t>(i) * n + col] = v[i] / nr;
    ++col;
  };
  std::vector<double> a(n), b(n);
  for (int t = 0; t < n && col < n; ++t) {
    const int e = idx[t];
    if (mu2[e] > 1e-20 * top && col + 1 < n) {
      // skip vectors already inside the span of stored pairs
      for (int i = 0; i < n; ++i) a[i] = V[static_cast<size_t>(i) * n + e];
      double before = 0.0, after;
      for (double x : a) before += x * x;
      std::vector<double> tst(a);
      for (int c = 0; c < col; ++c) {
        double d = 0.0;
        for (int i = 0; i < n; ++i) d += Q[static_cast<size_t>(i) * n + c] * tst[i];
        for (int i = 0; i < n; ++i) tst[i] -= d * Q[static_cast<size_t>(i) * n + c];
      }
      after = 0.0;
      for (double x : tst) after += x * x;
      if (after < 0.25 * before) continue;  // partner of an already stored pair
      put(tst);
      const double mu = std::sqrt(mu2[e]);
      for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += Ct[static_cast<size_t>(i) * n + k] * Q[static_cast<size_t>(k) * n + col - 1];
        b[i] = s / mu;
      }
      put(b);
      F.kind[col - 2] = 0;
      F.kind[col - 1] = 1;
    }
  }
  // remaining (zero-mode) directions: complete with eigenvectors orthogonal to the pairs
  for (int t = 0; t < n && col < n; ++t) {
    const int e = idx[n - 1 - t];
    for (int i = 0; i < n; ++i) a[i] = V[static_cast<size_t>(i) * n + e];
    std::vector<double> tst(a);
    for (int c = 0; c < col; ++c) {
      double d = 0.0;
      for (int i = 0; i < n; ++i) d += Q[static_cast<size_t>(i) * n + c] * tst[i];
      for (int i = 0; i < n; ++i) tst[i] -= d * Q[static_cast<size_t>(i) * n + c];
    }
    double nn = 0.0;
    for (double x : tst) nn += x * x;
    if (nn < 0.25) continue;
    put(tst);
    F.kind[col - 1] = 2;
  }
  if (col != n) { err = "time eigendecomposition failed"; return false; }
  // block values D = Q^T C Q
  F.mu.assign(n, 0.0);
  for (int c = 0; c < n; ++c) {
    if (F.kind[c] != 0) continue;
    double s = 0.0;
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k)
        s += Q[static_cast<size_t>(i) * n + c] * Ct[static_cast<size_t>(i) * n + k] * Q[static_cast<size_t>(k) * n + c + 1];
    F.mu[c] = s;        // D[c][c+1]
    F.mu[c + 1] = -s;   // D[c+1][c]
  }
  // Uo = L^{-T} Q
  std::vector<double> Uo(Q);
  upper_solve_T(L, n, Uo, n);
  // arrow completion: Mo v = -m, [t; rho] = [v; 1] / ||[v; 1]||_{M_t}
  std::vector<double> v(m);
  for (double& x : v) x = -x;
  lower_solve(L, n, v, 1);
  upper_solve_T(L, n, v, 1);
  std::vector<double> tv(N);
  for (int i = 0; i < n; ++i) tv[i] = v[i];
  tv[n] = 1.0;
  double nrm = 0.0;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) nrm += tv[i] * Mt[static_cast<size_t>(i) * N + j] * tv[j];
  nrm = std::sqrt(nrm);
  for (double& x : tv) x /= nrm;
  F.U.assign(static_cast<size_t>(N) * N, 0.0);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) F.U[static_cast<size_t>(i) * N + j] = Uo[static_cast<size_t>(i) * n + j];
    F.U[static_cast<size_t>(i) * N + n] = tv[i];
  }
  F.U[static_cast<size_t>(n) * N + n] = tv[n];
  // l = Uo^T (Wo t + w rho), sigma = [t; rho]^T W_t [t; rho]
  std::vector<double> g(n);
  for (int i = 0; i < n; ++i) {
    double s = w[i] * tv[n];
    for (int j = 0; j < n; ++j) s += Wo[static_cast<size_t>(i) * n + j] * tv[j];
    g[i] = s;
  }
  F.l.assign(n, 0.0);
  for (int c = 0; c < n; ++c) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += Uo[static_cast<size_t>(i) * n + c] * g[i];
    F.l[c] = s;
  }
  double sg = 0.0;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) sg += tv[i] * Wt[static_cast<size_t>(i) * N + j] * tv[j];
  F.sigma = sg;
  return true;
}

Gather banded_table(const std::vector<double>& A, int n, int row0, int nrow, int bw) {
  // rows row0 .. row0+nrow-1 of the full n x n matrix A; columns are full indices
  Gather G;
  G.n_out = nrow;
  G.W = 2 * bw + 1;
  G.col.assign(static_cast<size_t>(nrow) * G.W, 0);
  G.coef.assign(static_cast<size_t>(nrow) * G.W, 0.0);
  for (int r = 0; r < nrow; ++r) {
    const int i = row0 + r;
    for (int w = 0; w < G.W; ++w) {
      const int j = i - bw + w;
      const size_t o = static_cast<size_t>(r) * G.W + w;
      if (j < 0 || j >= n) { G.col[o] = i; G.coef[o] = 0.0; continue; }
      G.col[o] = j;
      G.coef[o] = A[static_cast<size_t>(i) * n + j];
    }
  }
  return G;
}

Gather eval_table(const Dir1D& D, int der) {
  Gather G;
  G.n_out = D.Q;
  G.W = D.p + 1;
  G.col.resize(static_cast<size_t>(D.Q) * G.W);
  G.coef.resize(static_cast<size_t>(D.Q) * G.W);
  for (int q = 0; q < D.Q; ++q)
    for (int j = 0; j <= D.p; ++j) {
      G.col[static_cast<size_t>(q) * G.W + j] = D.first[q] + j;
      G.coef[static_cast<size_t>(q) * G.W + j] = D.B[der][static_cast<size_t>(q) * (D.p + 1) + j];
    }
  return G;
}

Gather eval_table_T(const Dir1D& D, int der, const std::vector<double>* ws) {
  std::vector<std::vector<std::pair<int, double>>> rows(D.n);
  for (int q = 0; q < D.Q; ++q)
    for (int j = 0; j <= D.p; ++j)
      rows[D.first[q] + j].emplace_back(q, D.B[der][static_cast<size_t>(q) * (D.p + 1) + j] * (ws ? (*ws)[q] : 1.0));
  Gather G;
  G.n_out = D.n;
  G.W = 0;
  for (auto& r : rows) G.W = std::max(G.W, static_cast<int>(r.size()));
  G.col.assign(static_cast<size_t>(D.n) * G.W, 0);
  G.coef.assign(static_cast<size_t>(D.n) * G.W, 0.0);
  for (int i = 0; i < D.n; ++i)
    for (size_t k = 0; k < rows[i].size(); ++k) {
      G.col[static_cast<size_t>(i) * G.W + k] = rows[i][k].first;
      G.coef[static_cast<size_t>(i) * G.W + k] = rows[i][k].second;
    }
  // pad with a valid column of the row (weight 0)
  for (int i = 0; i < D.n; ++i)
    for (int k = static_cast<int>(rows[i].size()); k < G.W; ++k)
      G.col[static_cast<size_t>(i) * G.W + k] = rows[i].empty() ? 0 : rows[i][0].first;
  return G;
}

Gather streamline_table_T(const Dir1D& D, const std::vector<double>& tau) {
  Gather G = eval_table_T(D, 0, nullptr);
  // same rows and columns as the value projection; coefficients b + tau b'
  std::vector<int> fill(D.n, 0);
  for (int q = 0; q < D.Q; ++q)
    for (int j = 0; j <= D.p; ++j) {
      const int i = D.first[q] + j;
      const size_t k = static_cast<size_t>(i) * G.W + fill[i]++;
      G.coef[k] = D.B[0][static_cast<size_t>(q) * (D.p + 1) + j] + tau[q] * D.B[1][static_cast<size_t>(q) * (D.p + 1) + j];
    }
  return G;
}

Gather dense_table(const std::vector<double>& A, int nrow, int ncol, bool transpose) {
  Gather G;
  const int no = transpose ? ncol : nrow, ni = transpose ? nrow : ncol;
  G.n_out = no;
  G.W = ni;
  G.col.resize(static_cast<size_t>(no) * ni);
  G.coef.resize(static_cast<size_t>(no) * ni);
  for (int i = 0; i < no; ++i)
    for (int j = 0; j < ni; ++j) {
      G.col[static_cast<size_t>(i) * ni + j] = j;
      G.coef[static_cast<size_t>(i) * ni + j] =
          transpose ? A[static_cast<size_t>(j) * ncol + i] : A[static_cast<size_t>(i) * ncol + j];
    }
  return G;
}

void make_contiguous(Gather& G, int n_in) {
  G.c0.clear();
  const int W = G.W;
  if (W <= 0 || W > n_in) return;
  std::vector<int> c0(G.n_out);
  std::vector<int> col(G.col.size());
  std::vector<double> coef(G.coef.size(), 0.0);
  for (int i = 0; i < G.n_out; ++i) {
    int lo = n_in, hi = -1;
    for (int w = 0; w < W; ++w) {
      const size_t o = static_cast<size_t>(i) * W + w;
      if (G.coef[o] == 0.0) continue;
      lo = std::min(lo, G.col[o]);
      hi = std::max(hi, G.col[o]);
    }
    if (hi < 0) lo = hi = (i > 0 ? c0[i - 1] : 0);
    if (hi - lo + 1 > W) return;                       // not representable
    int start = std::min(std::max(lo, 0), n_in - W);
    if (start > lo) start = lo;                        // keep every non-zero inside the window
    if (i > 0 && start < c0[i - 1]) start = std::min(c0[i - 1], lo);
    if (start + W - 1 < hi || start < 0) return;
    c0[i] = start;
    for (int w = 0; w < W; ++w) col[static_cast<size_t>(i) * W + w] = start + w;
    for (int w = 0; w < W; ++w) {
      const size_t o = static_cast<size_t>(i) * W + w;
      if (G.coef[o] == 0.0) continue;
      coef[static_cast<size_t>(i) * W + (G.col[o] - start)] += G.coef[o];
    }
  }
  for (int i = 1; i < G.n_out; ++i)
    if (c0[i] < c0[i - 1]) return;                     // windows must not move backwards
  G.col = col;
  G.coef = coef;
  G.c0 = c0;
}

void hat_weights(const std::vector<double>& nodes, const std::vector<double>& x, std::vector<int>& left,
                 std::vector<double>& wl) {
  const int N = static_cast<int>(nodes.size());
  left.resize(x.size());
  wl.resize(x.size());
  for (size_t m = 0; m < x.size(); ++m) {
    if (N == 1 || x[m] <= nodes[0]) { left[m] = 0; wl[m] = 1.0; continue; }
    if (x[m] >= nodes[N - 1]) { left[m] = N - 2; wl[m] = 0.0; continue; }
    int g = static_cast<int>(std::upper_bound(nodes.begin(), nodes.end(), x[m]) - nodes.begin()) - 1;
    g = std::min(std::max(g, 0), N - 2);
    left[m] = g;
    wl[m] = (nodes[g + 1] - x[m]) / (nodes[g + 1] - nodes[g]);
  }
}

void support_windows(const Dir1D& D, int first, std::vector<int>& e0, std::vector<int>& e1) {
  const int nk = static_cast<int>(D.knots.size());
  e0.clear();
  e1.clear();
  for (int j = first; j < D.n; ++j) {
    const double lo = D.knots[std::max(j - D.p, 0)];
    const double hi = D.knots[std::min(j + D.p + 1, nk - 1)];
    int a = -1, b = -1;
    for (int e = 0; e < D.nel; ++e)
      if (D.brk[e] >= lo && D.brk[e + 1] <= hi) {
        if (a < 0) a = e;
        b = e + 1;
      }
    e0.push_back(a);
    e1.push_back(b);
  }
}

}  // namespace stiga
