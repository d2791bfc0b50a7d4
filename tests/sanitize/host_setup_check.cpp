// Driver for the sanitizer build of the host-side setup (AddressSanitizer +
// UndefinedBehaviorSanitizer, CPU only): runs every host routine of
// host_setup.cpp on uniform, graded, repeated-knot and mapped knot vectors of
// degrees 1..3 and checks a few invariants (partition of unity, mass sums,
// eigen-decomposition residuals), so that an out-of-bounds access or an
// undefined operation in the setup aborts the run.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "../../paper_2311_17500_amd/csrc/host_setup.hpp"

using namespace stiga;

static int failures = 0;
static void check(bool ok, const char* what, int p, int nel) {
  if (!ok) {
    std::printf("FAIL %s (p=%d nel=%d)\n", what, p, nel);
    ++failures;
  }
}

static std::vector<double> knots(int nel, int p, int kind) {
  std::vector<double> k(p + 1, 0.0);
  for (int i = 1; i < nel; ++i) {
    double x = static_cast<double>(i) / nel;
    if (kind == 1) x = x * x;                         // graded
    k.push_back(x);
    if (kind == 2 && i == nel / 2 && p > 1) k.push_back(x);   // a double interior knot
  }
  for (int i = 0; i <= p; ++i) k.push_back(1.0);
  return k;
}

int main() {
  for (int p = 1; p <= 3; ++p) {
    for (int nel : {1, 2, 5, 17}) {
      for (int kind = 0; kind < 3; ++kind) {
        std::vector<double> kn = knots(nel, p, kind);
        for (int mapk = 0; mapk < 3; ++mapk) {
          Dir1D D;
          std::string err;
          const bool ok = build_dir(kn.data(), static_cast<int>(kn.size()), p, 1.0, 2, D, err);
          check(ok, "build_dir", p, nel);
          if (!ok) continue;
          const double prm[3] = {-0.5, 1.5, mapk == 2 ? 2.0 : 0.0};
          check(apply_map(D, mapk, prm, err), "apply_map", p, nel);
          const double len = mapk == 0 ? 1.0 : 2.0;
          std::vector<double> M = gram1d(D, 0, 0, nullptr), K = gram1d(D, 1, 1, nullptr), Wm = gram1d(D, 0, 1, nullptr);
          double msum = 0.0, krow = 0.0;
          for (int i = 0; i < D.n; ++i) {
            double r = 0.0;
            for (int j = 0; j < D.n; ++j) {
              msum += M[static_cast<size_t>(i) * D.n + j];
              r += K[static_cast<size_t>(i) * D.n + j];
            }
            krow = std::max(krow, std::fabs(r));
          }
          // the graded map integrates an exponential with the (p + 1)-point rule: exact only in the limit
          check(std::fabs(msum - len) < (mapk == 2 ? 5e-2 : 1e-12), "mass sum", p, nel);
          check(krow < 1e-9 * (1.0 + nel * nel), "stiffness kernel", p, nel);
          std::vector<double> U, lam;
          if (D.n >= 2) check(gen_eig_sym(K, M, D.n, U, lam, err), "gen_eig_sym", p, nel);
          std::vector<double> Q, lq;
          check(sym_eig(M, D.n, Q, lq, err), "sym_eig", p, nel);
          Gather Mt = banded_table(M, D.n, 0, D.n, p), E0 = eval_table(D, 0), E2 = eval_table(D, 2);
          Gather ET = eval_table_T(D, 0, nullptr), DT = dense_table(M, D.n, D.n, true);
          make_contiguous(Mt, D.n);
          make_contiguous(E0, D.n);
          make_contiguous(ET, D.Q);
          std::vector<int> left, e0, e1;
          std::vector<double> wl;
          hat_weights(D.grev_x, D.xq, left, wl);
          support_windows(D, 0, e0, e1);
          std::vector<double> C = collocation(D, D.grev, 0);
          for (int i = 0; i < D.n; ++i) {
            double s = 0.0;
            for (int j = 0; j < D.n; ++j) s += C[static_cast<size_t>(i) * D.n + j];
            check(std::fabs(s - 1.0) < 1e-13, "partition of unity", p, nel);
          }
          (void)Wm;
          (void)DT;
          (void)E2;
        }
        // time direction: the fast-diagonalization data, the SUPG streamline
        // projection (any knots, repeated ones included) and tau (maximal
        // regularity only)
        Dir1D T;
        std::string err;
        if (!build_dir(kn.data(), static_cast<int>(kn.size()), p, 2.0, p, T, err)) continue;
        if (kind != 2) {
          std::vector<double> tauq, coefs;
          check(tau_at_quad(T, tauq, coefs, err), "tau_at_quad", p, nel);
        }
        {
          std::vector<double> tq(T.Q);
          for (int q = 0; q < T.Q; ++q) tq[q] = (T.brk[q / T.nq + 1] - T.brk[q / T.nq]) / (2.0 * p + 1.0);
          Gather SP = streamline_table_T(T, tq);
          make_contiguous(SP, T.Q);
          std::vector<double> Kt = gram1d(T, 1, 1, &tq), Wt = gram1d(T, 1, 0, &tq);
          double sk = 0.0;
          for (double v : Kt) sk += v;
          check(std::fabs(sk) < 1e-9 * (1.0 + nel), "tau-weighted time stiffness kernel", p, nel);
          (void)Wt;
        }
        const int nt = T.n, Nt = nt - 1;
        if (Nt < 2) continue;
        std::vector<double> Wf = gram1d(T, 0, 1, nullptr), Mf = gram1d(T, 0, 0, nullptr);
        std::vector<double> Wx(static_cast<size_t>(Nt) * Nt), Mx(static_cast<size_t>(Nt) * Nt);
        for (int i = 0; i < Nt; ++i)
          for (int j = 0; j < Nt; ++j) {
            Wx[static_cast<size_t>(i) * Nt + j] = Wf[static_cast<size_t>(i + 1) * nt + j + 1];
            Mx[static_cast<size_t>(i) * Nt + j] = Mf[static_cast<size_t>(i + 1) * nt + j + 1];
          }
        TimeFD fd;
        check(time_fd(Wx, Mx, Nt, fd, err), "time_fd", p, nel);
      }
    }
  }
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
