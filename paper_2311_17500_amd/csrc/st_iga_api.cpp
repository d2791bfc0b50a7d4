// C ABI of the space-time SU isogeometric solver (declared in include/st_iga.h).
//
// Host code orchestrates gfx950 kernels on the caller's stream; all device
// memory is carved from the caller's workspace.  See kernels.hip for the
// kernels and host_setup.cpp for the FP64 setup of the 1D data.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/st_iga.h"
#include "host_setup.hpp"
#include "kernels.hpp"

using namespace stiga;

namespace {

struct Fail {
  st_iga_status st;
  std::string msg;
};

#define CK(call)                                                                       \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) throw Fail{ST_IGA_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

void check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Fail{ST_IGA_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e)};
}

// Bump allocator over the caller's workspace; in dry mode it only measures.
struct Arena {
  char* base = nullptr;
  size_t cap = 0, off = 0;
  bool dry = true;
  void* take(size_t bytes) {
    off = (off + 255) & ~static_cast<size_t>(255);
    void* p = dry ? nullptr : base + off;
    off += bytes;
    if (!dry && off > cap) throw Fail{ST_IGA_ENOMEM, "workspace too small"};
    return p;
  }
  template <class T>
  T* get(int64_t n) { return static_cast<T*>(take(static_cast<size_t>(std::max<int64_t>(n, 1)) * sizeof(T))); }
};

// A table resident on the device in FP64 and FP32.
struct Tab {
  Gather h;
  DTable<double> d;
  DTable<float> f;
};

template <class C>
struct Prec;   // per-precision device data of the operators
}  // namespace

struct st_iga_ctx {
  st_iga_problem P{};
  st_iga_options opt{};
  int d = 0;
  std::vector<Dir1D> dir;   // d spatial + time (last)
  int n[3] = {1, 1, 1}, Q[3] = {1, 1, 1};
  int nt = 0, Nt = 0, nqt = 0, nelt = 0, nel[3] = {1, 1, 1};
  int NtP = 0;   // row stride of the low-rank time tables (N_t plus zero rows)
  int fd_np = 0; // leading 2x2 blocks of the time FD (the rest are 1x1 zero blocks)
  int64_t Ns = 0, Qs = 0, nunk = 0, nfull = 0, Nels = 0;
  int chunk_el = 1;
  int64_t big_len = 0;
  int slab = 1;
  int64_t slab_layers = 1;
  // mass and stiffness tables of an axis (index d: the time tables W_t, M_t)
  // share their windows, so one dual sweep applies both
  bool dual[4] = {false, false, false, false};
  // fused coefficient kernel along the slowest spatial axis (d >= 2)
  bool cf = false;
  int cf_slab = 1, cf_nchunk = 1;
  std::vector<double> cf_Bl_h;
  std::vector<int> cf_first_h, cf_chunks_h;
  double* cf_Bl_d = nullptr;
  float* cf_Bl_f = nullptr;
  // fused quadrature pass along the same axis: second derivatives there and
  // time elements per chunk
  bool qf = false;
  int qf_ne = 1;
  std::vector<double> cf_B2_h, qf_win_h, qf_wd_h;
  double *cf_B2_d = nullptr, *qf_win = nullptr, *qf_wd = nullptr;
  bool qf_x2 = false;   // 3D: the fused quadrature kernel forms the x2 expansion itself
  int *cf_first = nullptr, *cf_chunks = nullptr;
  Arena ar;
  std::string err;
  // host setup results
  std::vector<double> Mt_full, Wt_full, tauq, lam_s_h;
  std::vector<std::vector<double>> Us_h, lam_h;
  TimeFD fd;
  // tables
  Tab Ms[3], Ks[3], Bq[3][3], BqT[3], Hs[3], Gs[3], Us[3], UsT[3];
  Tab Mt_x, Wt_x, Bt0, Bt1, BtT, Gt, Ut, UtT;
  // zero-padded dense FD matrices for the MFMA mode products (A[i][j] applied as sum_j A[i][j] x_j)
  struct Dense {
    std::vector<double> h;
    double* d = nullptr;
    float* f = nullptr;
    bf16* b = nullptr;     // BF16 copy (BF16 mode: the mode products run on the BF16 MFMA)
    int n = 0, npad = 0;
  } DUsT[3], DUs[3], DUtT, DUt;
  // the w-update as one dense product along time (FP64 MFMA): the n_t x n_t
  // matrix whose first row (the initial layer, w = 0) is zero
  Dense DEw;
  // device data
  double *lam_d = nullptr, *mu_d = nullptr, *l_d = nullptr;
  float *lam_f = nullptr, *mu_f = nullptr, *l_f = nullptr;
  int* kind_d = nullptr;
  int *el_t_s = nullptr, *el_t_c = nullptr, *el_s_s[3] = {}, *el_s_c[3] = {};
  int *win_t_s = nullptr, *win_t_c = nullptr, *win_s_s[3] = {}, *win_s_c[3] = {};
  double *wq_s = nullptr, *wq_t = nullptr;
  double *xq_dev[3] = {nullptr, nullptr, nullptr}, *tq_dev = nullptr;   // Gauss abscissae
  Source src;                       // source term f of eq. (3.1) (kind 0: none)
  // fixed-point scheme of Section 3.1 (outer = 2): M_R with the exact C_r at
  // every space-time Gauss point (Cq, Gauss weights included) instead of a
  // low rank; per full time row the time elements of its support (re0/re1)
  bool exact_react = false;
  double* Cq_d = nullptr;
  float* Cq_f = nullptr;
  double* cq_out = nullptr;         // set while a quadrature pass must fill Cq_d
  int *re0 = nullptr, *re1 = nullptr;
  std::vector<int> re0_h, re1_h;
  // SUPG + shock capturing (su = 2): test functions v + tau v_t, tau =
  // h/(2 p_t + 1) per time element.  Ls[l]: 1D matrices int B_j'' B_i of the
  // strong-form diffusion; Wtau_x: time table sum_e tau_e int b_j b_i'; BtTs
  // and Bts: projection onto / values of b_i + tau b_i' at the time Gauss
  // points; scfac: sc_c h^2/4 per time Gauss point; Rq: the shock-capturing
  // coefficient at every Gauss point (Gauss weights included)
  bool supg = false, sc_on = false;
  bool dualL[3] = {false, false, false};
  Tab Ls[3], Wtau_x, BtTs;
  std::vector<double> Bts_h, scfac_h;
  double *Bts_d = nullptr, *scfac_d = nullptr;
  float* Bts_f = nullptr;
  double* Rq_d = nullptr;
  float* Rq_f = nullptr;
  double* rq_out = nullptr;         // set while a quadrature pass must fill Rq_d
  // preconditioner of the SUPG system: fast diagonalization in space, and
  // per spatial mode an exact banded solve in time with T_j = A + lam_j B,
  // B = M_t + W_tau, A = C_m (W_t + K_t^tau) plus the reaction and
  // shock-capturing terms with their spatial means at each time Gauss point
  // (refactorized at every linearization)
  bool banded = false;              // time part of the preconditioner: banded LU per spatial mode
  std::vector<double> timeA0_full, band_B_h, tq_h, wsum_h;
  // time profiles of the preconditioner at the time Gauss points: spatial
  // means of the reaction coefficient, of the shock-capturing coefficient and
  // of theta (empty: zero)
  std::vector<double> prof_cr, prof_sc, prof_th;
  double *bandA_d = nullptr, *bandB_d = nullptr, *bandF_d = nullptr, *rowsum_d = nullptr;
  float* bandF_f = nullptr;
  // low-rank factors
  int maxR = 0, Rth = 0, Rc = 0;
  double lr_relerr = 0.0;              // achieved relative Frobenius error of the last truncated SVD
  bool lr_capped = false;              // its rank was cut to max_rank (tolerance missed)
  double err_th = 0.0, err_c = 0.0;    // the same for the current theta and reaction factors
  bool cap_th = false, cap_c = false;
  std::vector<double> Uth_h, sth_h, Uc_h, sc_h;  // host copies: U (N_t x R), s
  double *Vth = nullptr, *Vc = nullptr;          // device N_s x maxR
  double *Psi = nullptr, *Tr = nullptr;
  float *Psi_f = nullptr, *Tr_f = nullptr;
  bool linearized = false;
  // buffers
  double *t4[4] = {}, *big[2] = {};
  float *t4f[4] = {}, *bigf[2] = {}, *xf = nullptr, *yf = nullptr;
  bf16 *t4b[4] = {}, *xb = nullptr, *yb = nullptr;
  void *Vb = nullptr, *Zb = nullptr;
  int64_t ldb = 0;   // column stride of Vb, Zb (elements)
  // HIP graphs of the Arnoldi steps (preconditioner, operator, Gram-Schmidt),
  // one per basis column and basis precision, valid for the ranks they were
  // captured with
  struct StepGraph {
    hipGraphExec_t exec = nullptr;
    int rth = -1, rc = -1;
  };
  std::vector<StepGraph> graphs[4];   // [basis FP64, FP32] x [two passes, delayed second pass]
  // stream the Krylov operators launch on: the caller's stream, or the
  // library's capture stream while a step graph is recorded (work cannot be
  // captured on the null stream)
  hipStream_t op_stream = nullptr, cap_stream = nullptr;
  // pinned host copies of two Arnoldi steps' scalars and the events that
  // mark their arrival (the next step may run meanwhile)
  double* step_host = nullptr;
  hipEvent_t step_ev[2] = {nullptr, nullptr};
  ~st_iga_ctx() {
    for (auto& v : graphs)
      for (auto& g : v)
        if (g.exec) hipGraphExecDestroy(g.exec);
    if (cap_stream) hipStreamDestroy(cap_stream);
    for (auto& e : step_ev)
      if (e) hipEventDestroy(e);
    if (step_host) hipHostFree(step_host);
  }
  int device = -1;                  // device current at setup
  bool noalloc_ok = false;          // the allocation-free scratch of that device is resolved
  std::string noalloc_err;
  int last_refinements = 0;
  double *rk = nullptr, *xk = nullptr, *wk = nullptr, *dk = nullptr, *bk = nullptr;
  double *VT = nullptr, *sol_rhs = nullptr, *sol_dx = nullptr;
  const double *rfull_u = nullptr, *rfull_w = nullptr;   // (u, w) whose ionic residual part is in rfull
  double *grid = nullptr, *grid2 = nullptr, *E = nullptr, *rfull = nullptr, *Cg = nullptr;
  double *part = nullptr, *dsc = nullptr, *gram = nullptr, *tmpR = nullptr;
  double* givens = nullptr;   // Givens state of the FGMRES cycle with the delayed second pass
  int nb_red = 0, nb_part = 0, gram_nb = 0;
};

namespace {

// ------------------------------------------------------------------ host setup
void validate(const st_iga_problem* P, const st_iga_options* O) {
  if (!P || !O) throw Fail{ST_IGA_EINVAL, "null problem or options"};
  if (P->d < 1 || P->d > 3) throw Fail{ST_IGA_EINVAL, "d must be 1, 2 or 3"};
  if (P->p_s < 1 || P->p_t < 1) throw Fail{ST_IGA_EINVAL, "degrees must be >= 1"};
  if (P->p_t > 5) throw Fail{ST_IGA_EINVAL, "time degree above 5 is not supported"};
  if (!(P->T > 0) || !(P->Cm > 0)) throw Fail{ST_IGA_EINVAL, "T and Cm must be positive"};
  for (int l = 0; l < P->d; ++l)
    if (!(P->sigma[l] > 0)) throw Fail{ST_IGA_EINVAL, "sigma must be positive"};
  if (!(P->a > 0) || !(P->b > 0) || !(P->de > 0) || P->c1 < 0 || P->c2 < 0)
    throw Fail{ST_IGA_EINVAL, "Rogers-McCulloch parameters out of range"};
  for (int l = 0; l <= P->d; ++l)
    if (!P->knots[l]) throw Fail{ST_IGA_EINVAL, "null knot vector"};
  if (O->restart < 1 || O->restart > 64) throw Fail{ST_IGA_EINVAL, "restart must be in 1..64"};
  if (O->graphs < 0 || O->graphs > 2) throw Fail{ST_IGA_EINVAL, "graphs must be 0, 1 or 2"};
  if (O->reorth < 0 || O->reorth > 2) throw Fail{ST_IGA_EINVAL, "reorth must be 0, 1 or 2"};
  if (O->outer < 0 || O->outer > 2) throw Fail{ST_IGA_EINVAL, "outer must be 0, 1 or 2"};
  if (O->stall_cycles < 0 || !(O->stall_reduction >= 0.0 && O->stall_reduction < 1.0))
    throw Fail{ST_IGA_EINVAL, "stall_cycles >= 0 and 0 <= stall_reduction < 1 required"};
  if (O->picard_switch < 0) throw Fail{ST_IGA_EINVAL, "picard_switch must be >= 0"};
  if (!(O->alpha > 0) || O->alpha > 1) throw Fail{ST_IGA_EINVAL, "alpha must be in (0, 1]"};
  if (O->max_rank < 1 || O->max_rank > 128) throw Fail{ST_IGA_EINVAL, "max_rank must be in 1..128"};
  if (O->prec < ST_IGA_FP64 || O->prec > ST_IGA_MIXED_BF16) throw Fail{ST_IGA_EINVAL, "bad precision"};
  if (O->su < 0 || O->su > 2) throw Fail{ST_IGA_EINVAL, "su must be 0, 1 or 2"};
  if (O->su == 2 && O->outer != 2)
    throw Fail{ST_IGA_EINVAL, "SUPG + shock capturing (su = 2) runs in the fixed-point scheme (outer = 2)"};
  if (!(O->sc_c >= 0.0) || !std::isfinite(O->sc_c)) throw Fail{ST_IGA_EINVAL, "sc_c must be finite and >= 0"};
  if (O->precond < 0 || O->precond > 1) throw Fail{ST_IGA_EINVAL, "precond must be 0 or 1"};
  if (O->precond == 1 && O->su != 2 && !(P->a * P->c1 > 0.0))
    throw Fail{ST_IGA_EINVAL, "the banded time solve (precond = 1) needs a reaction shift a*c1 > 0 "
                              "(its factorization has no pivoting)"};
  if (O->su == 1) {  // SU needs C^{p_t - 1} in time: interior time multiplicity 1
    const double* k = P->knots[P->d];
    const int nk = P->nknots[P->d];
    for (int i = P->p_t + 1; i + 1 <= nk - P->p_t - 2; ++i)   // interior knots only
      if (k[i] == k[i + 1]) throw Fail{ST_IGA_EINVAL, "SU needs maximal time regularity"};
  }
}

std::vector<double> sub_rows(const std::vector<double>& A, int n, int r0, int r1, int c0, int c1) {
  std::vector<double> B(static_cast<size_t>(r1 - r0) * (c1 - c0));
  for (int i = r0; i < r1; ++i)
    for (int j = c0; j < c1; ++j) B[static_cast<size_t>(i - r0) * (c1 - c0) + (j - c0)] = A[static_cast<size_t>(i) * n + j];
  return B;
}

Gather sparse_rows(const std::vector<double>& A, int nrow, int ncol) {
  Gather G;
  G.n_out = nrow;
  G.W = 1;
  for (int i = 0; i < nrow; ++i) {
    int c = 0;
    for (int j = 0; j < ncol; ++j) c += A[static_cast<size_t>(i) * ncol + j] != 0.0;
    G.W = std::max(G.W, c);
  }
  G.col.assign(static_cast<size_t>(nrow) * G.W, 0);
  G.coef.assign(static_cast<size_t>(nrow) * G.W, 0.0);
  for (int i = 0; i < nrow; ++i) {
    int k = 0;
    for (int j = 0; j < ncol; ++j)
      if (A[static_cast<size_t>(i) * ncol + j] != 0.0) {
        G.col[static_cast<size_t>(i) * G.W + k] = j;
        G.coef[static_cast<size_t>(i) * G.W + k] = A[static_cast<size_t>(i) * ncol + j];
        ++k;
      }
    for (; k < G.W; ++k) G.col[static_cast<size_t>(i) * G.W + k] = 0;
  }
  return G;
}

Gather hat_table(const std::vector<double>& nodes, const std::vector<double>& x) {
  std::vector<int> left;
  std::vector<double> wl;
  hat_weights(nodes, x, left, wl);
  Gather G;
  G.n_out = static_cast<int>(x.size());
  G.W = 2;
  G.col.resize(x.size() * 2);
  G.coef.resize(x.size() * 2);
  const int N = static_cast<int>(nodes.size());
  for (size_t m = 0; m < x.size(); ++m) {
    G.col[2 * m] = left[m];
    G.coef[2 * m] = wl[m];
    G.col[2 * m + 1] = std::min(left[m] + 1, N - 1);
    G.coef[2 * m + 1] = (N == 1) ? 0.0 : 1.0 - wl[m];
  }
  return G;
}

// Plan of the fused coefficient kernel along the slowest spatial axis: basis
// values at that axis' Gauss points, the first B-spline of each element,
// time slabs sized to the two scratch buffers (expanded arrays of the faster
// axes only) and, when columns x time slabs give too few threads for the
// device, a split of the axis into B-spline ranges walked independently.
void plan_fused_coef(st_iga_ctx* c) {
  const int d = c->d;
  c->cf = d >= 2 && c->P.p_s <= 4 && c->P.p_t <= 5;
  if (!c->cf) return;
  const Dir1D& D = c->dir[d - 1];
  const int kp = D.p + 1;
  if (D.nq != kp) {
    c->cf = false;
    return;
  }
  c->cf_Bl_h.assign(static_cast<size_t>(D.Q) * kp, 0.0);
  for (int q = 0; q < D.Q; ++q)
    for (int k = 0; k < kp; ++k) c->cf_Bl_h[static_cast<size_t>(q) * kp + k] = D.B[0][static_cast<size_t>(q) * kp + k];
  c->cf_first_h.resize(D.nel);
  for (int e = 0; e < D.nel; ++e) c->cf_first_h[e] = D.first[static_cast<size_t>(e) * D.nq];
  // per-layer footprint of the expanded arrays in each scratch buffer
  int64_t Qin = 1;
  for (int l = 0; l < d - 1; ++l) Qin *= c->Q[l];
  const int64_t nd = D.n;
  const int64_t fl = (d == 3) ? nd * c->n[1] * c->Q[0] + nd * Qin : nd * Qin;
  const int halo = 2 * c->P.p_t + 1;
  const int64_t fit = c->big_len / std::max<int64_t>(fl, 1) - halo;
  c->cf_slab = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(c->Nt, fit)));
  if (c->opt.coef_slab > 0) c->cf_slab = std::min(c->Nt, c->opt.coef_slab);
  if (static_cast<int64_t>(c->cf_slab + halo) * fl > c->big_len) {
    c->cf = false;
    return;
  }
  const int64_t threads = Qin * ((c->cf_slab + 7) / 8);
  const int64_t want = 1 << 19;
  int nch = static_cast<int>(std::min<int64_t>(std::max<int64_t>(1, (want + threads - 1) / threads),
                                               std::max(1, D.nel / 4)));
  nch = std::max(1, std::min(nch, D.n));
  c->cf_nchunk = nch;
  c->cf_chunks_h.assign(4 * static_cast<size_t>(nch), 0);
  for (int k = 0; k < nch; ++k) {
    const int d0 = static_cast<int>(static_cast<int64_t>(k) * D.n / nch);
    const int d1 = static_cast<int>(static_cast<int64_t>(k + 1) * D.n / nch);
    int e0 = D.nel, e1 = 0;
    for (int e = 0; e < D.nel; ++e) {
      const int f = c->cf_first_h[e];
      if (f + D.p >= d0 && f < d1) {   // element touches a B-spline of [d0, d1)
        e0 = std::min(e0, e);
        e1 = std::max(e1, e + 1);
      }
    }
    if (e0 >= e1) e0 = e1 = 0;
    c->cf_chunks_h[4 * k] = e0;
    c->cf_chunks_h[4 * k + 1] = e1;
    c->cf_chunks_h[4 * k + 2] = d0;
    c->cf_chunks_h[4 * k + 3] = d1;
  }
  // quadrature pass: per time element, the first buffer holds the time
  // gathers (3 N_s per Gauss row) and, in 3D, the four x1 expansions; the
  // second holds the five inputs of the fused kernel, its projection output
  // and the element maxima before and after the x1 reduction
  c->cf_B2_h.assign(static_cast<size_t>(D.Q) * kp, 0.0);
  for (int q = 0; q < D.Q; ++q)
    for (int k = 0; k < kp; ++k) c->cf_B2_h[static_cast<size_t>(q) * kp + k] = D.B[2][static_cast<size_t>(q) * kp + k];
  const int nqt = c->nqt;
  const int64_t x1 = (d == 3) ? static_cast<int64_t>(c->n[2]) * c->n[1] * c->Q[0] : 0;
  const int64_t per0 = nqt * (3 * c->Ns + 4 * x1);
  const int64_t per1 = nqt * 6 * nd * Qin + 2LL * D.nel * Qin;
  const int64_t ne = std::min(c->big_len / per0, c->big_len / per1);
  c->qf = nqt >= 1 && nqt <= 6 && ne >= 1;
  // x2 value and second-derivative tables with the same contiguous in-range
  // windows of p + 1 B-splines: the quadrature kernel expands along x2 itself
  c->qf_x2 = false;
  if (d == 3) {
    const Gather &g0 = c->Bq[1][0].h, &g2 = c->Bq[1][2].h;
    bool ok = g0.W == kp && g2.W == kp && g0.n_out == c->Q[1] && g2.n_out == c->Q[1] &&
              static_cast<int>(g0.c0.size()) == c->Q[1] && g0.c0 == g2.c0;
    for (int q = 0; ok && q < c->Q[1]; ++q) ok = g0.c0[q] >= 0 && g0.c0[q] + kp <= c->n[1];
    c->qf_x2 = ok;
  }
  // spatial Gauss weights factored as (faster axes) x (this axis), each
  // product formed in the same order as the full tensor weights
  c->qf_win_h.assign(Qin, 1.0);
  for (int64_t q = 0; q < Qin; ++q) {
    int64_t r = q;
    double w = 1.0;
    for (int l = 0; l < d - 1; ++l) {
      w *= c->dir[l].wq[r % c->Q[l]];
      r /= c->Q[l];
    }
    c->qf_win_h[q] = w;
  }
  c->qf_wd_h = D.wq;
  c->qf_ne = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(c->nelt, ne)));
}

// Process-wide cache of the 1D eigen setups and of the SU coefficients tau_k.
// The pencils (K_l, M_l) and (W_t, M_t) and the tau_k depend only on knots,
// degree, map and T, not on sigma or the ionic parameters, so requests of the
// same shape (a serving stream repeats a few dozen shapes) share them.  Keyed by the exact matrix entries; at most
// kEigCacheMax entries of each kind (oldest evicted); thread-safe.
constexpr size_t kEigCacheMax = 32;
struct EigCache {
  std::mutex mu;
  std::map<std::vector<double>, std::pair<std::vector<double>, std::vector<double>>> space;   // -> (U, lambda)
  std::map<std::vector<double>, TimeFD> time;
  std::map<std::vector<double>, std::vector<double>> tau;   // time knots (+ degree) -> tau_k at the Gauss points
  std::vector<std::vector<double>> space_order, time_order, tau_order;
};
EigCache& eig_cache() {
  static EigCache c;
  return c;
}
std::vector<double> pencil_key(const std::vector<double>& A, const std::vector<double>& B, int n) {
  std::vector<double> k;
  k.reserve(A.size() + B.size() + 1);
  k.push_back(static_cast<double>(n));
  k.insert(k.end(), A.begin(), A.end());
  k.insert(k.end(), B.begin(), B.end());
  return k;
}
bool gen_eig_sym_cached(const std::vector<double>& K, const std::vector<double>& M, int n, std::vector<double>& U,
                        std::vector<double>& lam, std::string& err) {
  EigCache& c = eig_cache();
  const std::vector<double> key = pencil_key(K, M, n);
  {
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.space.find(key);
    if (it != c.space.end()) {
      U = it->second.first;
      lam = it->second.second;
      return true;
    }
  }
  if (!gen_eig_sym(K, M, n, U, lam, err)) return false;
  std::lock_guard<std::mutex> g(c.mu);
  if (c.space.emplace(key, std::make_pair(U, lam)).second) {
    c.space_order.push_back(key);
    if (c.space_order.size() > kEigCacheMax) {
      c.space.erase(c.space_order.front());
      c.space_order.erase(c.space_order.begin());
    }
  }
  return true;
}
bool time_fd_cached(const std::vector<double>& Wt, const std::vector<double>& Mt, int N, TimeFD& F,
                    std::string& err) {
  EigCache& c = eig_cache();
  const std::vector<double> key = pencil_key(Wt, Mt, N);
  {
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.time.find(key);
    if (it != c.time.end()) {
      F = it->second;
      return true;
    }
  }
  if (!time_fd(Wt, Mt, N, F, err)) return false;
  std::lock_guard<std::mutex> g(c.mu);
  if (c.time.emplace(key, F).second) {
    c.time_order.push_back(key);
    if (c.time_order.size() > kEigCacheMax) {
      c.time.erase(c.time_order.front());
      c.time_order.erase(c.time_order.begin());
    }
  }
  return true;
}

bool tau_at_quad_cached(const Dir1D& T, std::vector<double>& tauq, std::string& err) {
  EigCache& c = eig_cache();
  std::vector<double> key(T.knots);
  key.push_back(static_cast<double>(T.p));
  key.push_back(static_cast<double>(T.nq));
  {
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.tau.find(key);
    if (it != c.tau.end()) {
      tauq = it->second;
      return true;
    }
  }
  std::vector<double> coefs;
  if (!tau_at_quad(T, tauq, coefs, err)) return false;
  std::lock_guard<std::mutex> g(c.mu);
  if (c.tau.emplace(key, tauq).second) {
    c.tau_order.push_back(key);
    if (c.tau_order.size() > kEigCacheMax) {
      c.tau.erase(c.tau_order.front());
      c.tau_order.erase(c.tau_order.begin());
    }
  }
  return true;
}

// Band [t][2p+1] (column t - p + k, zero outside) of the X_t block
// (full rows and columns 1..nt-1) of a full nt x nt matrix.
std::vector<double> band_rows(const std::vector<double>& A, int nt, int p) {
  const int Nt = nt - 1, KW = 2 * p + 1;
  std::vector<double> b(static_cast<size_t>(Nt) * KW, 0.0);
  for (int t = 0; t < Nt; ++t)
    for (int k = 0; k < KW; ++k) {
      const int col = t - p + k;
      if (col >= 0 && col < Nt) b[static_cast<size_t>(t) * KW + k] = A[static_cast<size_t>(t + 1) * nt + col + 1];
    }
  return b;
}

void host_setup(st_iga_ctx* c) {
  const st_iga_problem& P = c->P;
  c->d = P.d;
  c->dir.assign(P.d + 1, Dir1D());
  std::string err;
  for (int l = 0; l < P.d; ++l) {
    if (!build_dir(P.knots[l], P.nknots[l], P.p_s, 1.0, 2, c->dir[l], err)) throw Fail{ST_IGA_EINVAL, "space knots: " + err};
    if (!apply_map(c->dir[l], P.map_kind[l], P.map_param[l], err)) throw Fail{ST_IGA_EINVAL, err};
  }
  if (!build_dir(P.knots[P.d], P.nknots[P.d], P.p_t, P.T, P.p_t, c->dir[P.d], err))
    throw Fail{ST_IGA_EINVAL, "time knots: " + err};
  const Dir1D& T = c->dir[P.d];
  // exact reaction (fixed-point scheme of Section 3.1): the time elements in
  // the support of each full time row
  c->exact_react = c->opt.outer == 2;
  if (c->exact_react) {
    c->re0_h.assign(T.n, T.nel);
    c->re1_h.assign(T.n, 0);
    for (int e = 0; e < T.nel; ++e) {
      const int fe = T.first[static_cast<size_t>(e) * T.nq];
      for (int a = 0; a <= T.p; ++a) {
        const int i = fe + a;
        if (i < 0 || i >= T.n) continue;
        c->re0_h[i] = std::min(c->re0_h[i], e);
        c->re1_h[i] = std::max(c->re1_h[i], e + 1);
      }
    }
  }
  c->Ns = 1;
  c->Qs = 1;
  c->Nels = 1;
  for (int l = 0; l < P.d; ++l) {
    c->n[l] = c->dir[l].n;
    c->Q[l] = c->dir[l].Q;
    c->nel[l] = c->dir[l].nel;
    c->Ns *= c->n[l];
    c->Qs *= c->Q[l];
    c->Nels *= c->nel[l];
  }
  c->nt = T.n;
  c->Nt = T.n - 1;
  c->nqt = T.nq;
  c->nelt = T.nel;
  if (c->Nt < 2) throw Fail{ST_IGA_EINVAL, "need at least two time unknowns"};
  if (c->Nt > 142) throw Fail{ST_IGA_EINVAL, "more than 142 time unknowns is not supported"};
  c->nunk = c->Ns * c->Nt;
  c->nfull = c->Ns * c->nt;
  c->maxR = c->opt.max_rank;
  // 1D matrices
  c->Mt_full = gram1d(T, 0, 0, nullptr);
  c->Wt_full = gram1d(T, 0, 1, nullptr);
  const int nt = c->nt, Nt = c->Nt, pt = P.p_t;
  c->Mt_x.h = banded_table(c->Mt_full, nt, 1, Nt, pt);
  c->Wt_x.h = banded_table(c->Wt_full, nt, 1, Nt, pt);
  c->Bt0.h = eval_table(T, 0);
  c->Bt1.h = eval_table(T, 1);
  c->BtT.h = eval_table_T(T, 0, nullptr);
  // the tau_k of the SU term need C^{p_t - 1} time splines: SU only
  if (c->opt.su == 1) {
    if (!tau_at_quad_cached(T, c->tauq, err)) throw Fail{ST_IGA_EINVAL, err};
  } else {
    c->tauq.assign(static_cast<size_t>(pt) * T.Q, 0.0);
  }
  c->supg = c->opt.su == 2;
  c->sc_on = c->supg && c->opt.sc_c > 0.0;
  if (c->supg) {
    // Section 4.2.2: tau = h/(2p+1) and c h^2/4 with h the time element length
    std::vector<double> tq(T.Q);
    c->scfac_h.assign(T.Q, 0.0);
    c->Bts_h.assign(static_cast<size_t>(T.Q) * (pt + 1), 0.0);
    for (int q = 0; q < T.Q; ++q) {
      const int e = q / T.nq;
      const double h = T.brk[e + 1] - T.brk[e];
      tq[q] = h / (2.0 * pt + 1.0);
      c->scfac_h[q] = c->opt.sc_c * h * h / 4.0;
      for (int a = 0; a <= pt; ++a)
        c->Bts_h[static_cast<size_t>(q) * (pt + 1) + a] =
            T.B[0][static_cast<size_t>(q) * (pt + 1) + a] + tq[q] * T.B[1][static_cast<size_t>(q) * (pt + 1) + a];
    }
    // C_m (W_t + K_t^tau) on the mass part, W_tau on the strong-form diffusion
    std::vector<double> Wsum = c->Wt_full;
    const std::vector<double> Kt = gram1d(T, 1, 1, &tq);
    for (size_t k = 0; k < Wsum.size(); ++k) Wsum[k] += Kt[k];
    c->Wt_x.h = banded_table(Wsum, nt, 1, Nt, pt);
    const std::vector<double> Wtau = gram1d(T, 1, 0, &tq);
    c->Wtau_x.h = banded_table(Wtau, nt, 1, Nt, pt);
    c->BtTs.h = streamline_table_T(T, tq);
    c->tq_h = tq;
    c->timeA0_full = Wsum;
    for (double& v : c->timeA0_full) v *= P.Cm;
    std::vector<double> Bf = c->Mt_full;
    for (size_t k = 0; k < Bf.size(); ++k) Bf[k] += Wtau[k];
    c->band_B_h = band_rows(Bf, nt, pt);
  }
  c->banded = c->supg || c->opt.precond == 1;
  if (c->banded && !c->supg) {
    // A = C_m W_t (+ the profile terms at each linearization), B = M_t
    c->timeA0_full = c->Wt_full;
    for (double& v : c->timeA0_full) v *= P.Cm;
    c->band_B_h = band_rows(c->Mt_full, nt, pt);
  }
  c->Us_h.assign(P.d, {});
  c->lam_h.assign(P.d, {});
  for (int l = 0; l < P.d; ++l) {
    const Dir1D& D = c->dir[l];
    std::vector<double> M = gram1d(D, 0, 0, nullptr), K = gram1d(D, 1, 1, nullptr);
    c->Ms[l].h = banded_table(M, D.n, 0, D.n, D.p);
    c->Ks[l].h = banded_table(K, D.n, 0, D.n, D.p);
    if (c->supg) c->Ls[l].h = banded_table(gram1d(D, 0, 2, nullptr), D.n, 0, D.n, D.p);
    for (int k = 0; k <= 2; ++k) c->Bq[l][k].h = eval_table(D, k);
    c->BqT[l].h = eval_table_T(D, 0, nullptr);
    c->Hs[l].h = hat_table(D.grev_x, D.xq);   // interpolation at the mapped Greville abscissae
    c->Gs[l].h = sparse_rows(collocation(D, D.grev, 0), D.n, D.n);
    if (!gen_eig_sym_cached(K, M, D.n, c->Us_h[l], c->lam_h[l], err)) throw Fail{ST_IGA_EINVAL, err};
    c->Us[l].h = dense_table(c->Us_h[l], D.n, D.n, false);
    c->UsT[l].h = dense_table(c->Us_h[l], D.n, D.n, true);
  }
  // time Greville collocation on X_t Greville points
  std::vector<double> gt(T.grev.begin() + 1, T.grev.end());
  c->Gt.h = sparse_rows(collocation(T, gt, 0), Nt, nt);
  // FD time data on the X_t block
  std::vector<double> Wx = sub_rows(c->Wt_full, nt, 1, nt, 1, nt), Mx = sub_rows(c->Mt_full, nt, 1, nt, 1, nt);
  if (!time_fd_cached(Wx, Mx, Nt, c->fd, err)) throw Fail{ST_IGA_EINVAL, err};
  // the 2x2 blocks lead, 1x1 blocks follow (checked: the kernel relies on it)
  c->fd_np = 0;
  while (2 * c->fd_np + 1 < Nt - 1 && c->fd.kind[2 * c->fd_np] == 0 && c->fd.kind[2 * c->fd_np + 1] == 1) ++c->fd_np;
  for (int i = 2 * c->fd_np; i < Nt - 1; ++i)
    if (c->fd.kind[i] != 2) throw Fail{ST_IGA_EINVAL, "time fast diagonalization: unexpected block order"};
  c->Ut.h = dense_table(c->fd.U, Nt, Nt, false);
  c->UtT.h = dense_table(c->fd.U, Nt, Nt, true);
  auto pad = [](st_iga_ctx::Dense& D, const std::vector<double>& U, int n, bool transpose) {
    D.n = n;
    D.npad = 16 * ((n + 15) / 16);
    D.h.assign(static_cast<size_t>(D.npad) * D.npad, 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        D.h[static_cast<size_t>(i) * D.npad + j] = transpose ? U[static_cast<size_t>(j) * n + i] : U[static_cast<size_t>(i) * n + j];
  };
  if (Nt > 144) throw Fail{ST_IGA_EINVAL, "more than 144 time unknowns is not supported"};
  pad(c->DUt, c->fd.U, Nt, false);
  pad(c->DUtT, c->fd.U, Nt, true);
  for (int l = 0; l < P.d; ++l) {
    if (c->n[l] > 144) throw Fail{ST_IGA_EINVAL, "more than 144 basis functions per direction is not supported"};
    pad(c->DUs[l], c->Us_h[l], c->n[l], false);
    pad(c->DUsT[l], c->Us_h[l], c->n[l], true);
  }
  // spatial eigenvalue sums + shift
  c->lam_s_h.assign(c->Ns, 0.0);
  for (int64_t j = 0; j < c->Ns; ++j) {
    int64_t r = j;
    double s = P.a * P.c1;
    for (int l = 0; l < P.d; ++l) {
      const int il = static_cast<int>(r % c->n[l]);
      r /= c->n[l];
      s += P.sigma[l] * c->lam_h[l][il];
    }
    c->lam_s_h[j] = s;
  }
  // the 1x1 (zero-frequency) time blocks of the arrowhead divide by the
  // spatial shift a c1 + sum_l sigma_l lambda_l; with a c1 = 0 the constant
  // Neumann mode makes it (numerically) zero
  if (!c->banded && 2 * c->fd_np < Nt - 1) {   // (the banded time solve needs no such split)
    double smin = INFINITY, smax = 0.0;
    for (double v : c->lam_s_h) {
      smin = std::min(smin, std::fabs(v));
      smax = std::max(smax, std::fabs(v));
    }
    if (!(smin > 1e-12 * std::max(smax, 1.0)))
      throw Fail{ST_IGA_EINVAL, "fast-diagonalization preconditioner: a zero-frequency time block meets a spatial mode "
                                "with zero shift (a*c1 = 0 with Neumann boundaries and an odd N_t - 1); use c1 > 0 "
                                "or an even N_t - 1"};
  }
  // w-update operator: b (W + b de M)^{-1}_{XtXt} M_{Xt,full}
  {
    std::vector<double> L(static_cast<size_t>(Nt) * Nt), R(static_cast<size_t>(Nt) * nt);
    for (int i = 0; i < Nt; ++i) {
      for (int j = 0; j < Nt; ++j)
        L[static_cast<size_t>(i) * Nt + j] = c->Wt_full[static_cast<size_t>(i + 1) * nt + j + 1] +
                                             P.b * P.de * c->Mt_full[static_cast<size_t>(i + 1) * nt + j + 1];
      for (int j = 0; j < nt; ++j) R[static_cast<size_t>(i) * nt + j] = P.b * c->Mt_full[static_cast<size_t>(i + 1) * nt + j];
    }
    // Gaussian elimination with partial pivoting on [L | R]
    for (int col = 0; col < Nt; ++col) {
      int pr = col;
      for (int r = col + 1; r < Nt; ++r)
        if (std::fabs(L[static_cast<size_t>(r) * Nt + col]) > std::fabs(L[static_cast<size_t>(pr) * Nt + col])) pr = r;
      if (L[static_cast<size_t>(pr) * Nt + col] == 0.0) throw Fail{ST_IGA_EINVAL, "singular w-update matrix"};
      if (pr != col) {
        for (int k = 0; k < Nt; ++k) std::swap(L[static_cast<size_t>(col) * Nt + k], L[static_cast<size_t>(pr) * Nt + k]);
        for (int k = 0; k < nt; ++k) std::swap(R[static_cast<size_t>(col) * nt + k], R[static_cast<size_t>(pr) * nt + k]);
      }
      for (int r = 0; r < Nt; ++r) {
        if (r == col) continue;
        const double f = L[static_cast<size_t>(r) * Nt + col] / L[static_cast<size_t>(col) * Nt + col];
        if (f == 0.0) continue;
        for (int k = col; k < Nt; ++k) L[static_cast<size_t>(r) * Nt + k] -= f * L[static_cast<size_t>(col) * Nt + k];
        for (int k = 0; k < nt; ++k) R[static_cast<size_t>(r) * nt + k] -= f * R[static_cast<size_t>(col) * nt + k];
      }
    }
    for (int r = 0; r < Nt; ++r)
      for (int k = 0; k < nt; ++k) R[static_cast<size_t>(r) * nt + k] /= L[static_cast<size_t>(r) * Nt + r];
    // n_t <= 143 (checked above): at most nine 16-row tiles
    st_iga_ctx::Dense& D = c->DEw;
    D.n = nt;
    D.npad = 16 * ((nt + 15) / 16);
    D.h.assign(static_cast<size_t>(D.npad) * D.npad, 0.0);
    for (int r = 0; r < Nt; ++r)
      for (int k = 0; k < nt; ++k) D.h[static_cast<size_t>(r + 1) * D.npad + k] = R[static_cast<size_t>(r) * nt + k];
  }
  // chunking of the quadrature pass: arrays per time Gauss point row
  // contiguous windows for the sweep kernels
  for (int l = 0; l < P.d; ++l) {
    const Dir1D& D = c->dir[l];
    make_contiguous(c->Ms[l].h, D.n);
    make_contiguous(c->Ks[l].h, D.n);
    for (int k2 = 0; k2 <= 2; ++k2) make_contiguous(c->Bq[l][k2].h, D.n);
    make_contiguous(c->BqT[l].h, D.Q);
    make_contiguous(c->Hs[l].h, D.n);
    make_contiguous(c->Gs[l].h, D.n);
  }
  make_contiguous(c->Mt_x.h, c->nt);
  make_contiguous(c->Wt_x.h, c->nt);
  auto same_windows = [](const Gather& A, const Gather& B) {
    return !A.c0.empty() && A.c0 == B.c0 && A.W == B.W && A.n_out == B.n_out;
  };
  for (int l = 0; l < P.d; ++l) c->dual[l] = same_windows(c->Ms[l].h, c->Ks[l].h);
  c->dual[P.d] = same_windows(c->Mt_x.h, c->Wt_x.h);
  if (c->supg) {
    for (int l = 0; l < P.d; ++l) {
      make_contiguous(c->Ls[l].h, c->dir[l].n);
      c->dualL[l] = same_windows(c->Ms[l].h, c->Ls[l].h);
    }
    make_contiguous(c->Wtau_x.h, c->nt);
    make_contiguous(c->BtTs.h, T.Q);
  }
  make_contiguous(c->Bt0.h, c->nt);
  make_contiguous(c->Bt1.h, c->nt);
  make_contiguous(c->BtT.h, T.Q);
  make_contiguous(c->Gt.h, c->nt);
  // the quadrature pass keeps 3 arrays of N_s and 3 of Q_s doubles per time
  // Gauss point in the first big buffer and 5 of Q_s in the second
  // time slabs of the coefficient part: whole time axis unless the two
  // scratch buffers would exceed about 24 GB in FP64
  {
    const int64_t cap_layers = std::max<int64_t>(8, (int64_t(3) << 29) / std::max<int64_t>(c->Qs, 1));
    const int halo = 2 * c->P.p_t + 1;
    c->slab = (c->nt <= cap_layers) ? c->Nt : static_cast<int>(std::max<int64_t>(4, cap_layers - halo));
    if (c->opt.coef_slab > 0) c->slab = std::min(c->Nt, c->opt.coef_slab);
    c->slab_layers = std::min<int64_t>(c->nt, c->slab + halo);
  }
  c->big_len = std::max<int64_t>({c->slab_layers * c->Qs, 5LL * c->nqt * c->Qs,
                                  3LL * c->nqt * (c->Ns + c->Qs), 2LL * c->Qs + 0});
  const int64_t cq = std::min<int64_t>(c->big_len / (3 * (c->Ns + c->Qs)), c->big_len / (5 * c->Qs));
  c->chunk_el = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(c->nelt, cq / c->nqt)));
  plan_fused_coef(c);
}

// Reserve device memory for everything; in dry mode only sizes are computed.
template <class C>
void alloc_tab(Arena& a, Tab& t) {
  const size_t n = t.h.col.size();
  if (!t.h.c0.empty()) {
    t.d.c0 = a.get<int>(static_cast<int64_t>(t.h.c0.size()));
    t.f.c0 = t.d.c0;
  }
  t.d.col = a.get<int>(n);
  t.d.coef = a.get<double>(n);
  t.f.col = t.d.col;
  t.f.coef = a.get<float>(n);
  t.d.n_out = t.f.n_out = t.h.n_out;
  t.d.W = t.f.W = t.h.W;
}

void plan(st_iga_ctx* c) {
  Arena& a = c->ar;
  const bool mixed = c->opt.prec != ST_IGA_FP64;
  const bool bf = c->opt.prec == ST_IGA_MIXED_BF16;
  const int d = c->d;
  auto T = [&](Tab& t) { alloc_tab<double>(a, t); };
  for (int l = 0; l < d; ++l) {
    T(c->Ms[l]); T(c->Ks[l]); T(c->BqT[l]); T(c->Hs[l]); T(c->Gs[l]); T(c->Us[l]); T(c->UsT[l]);
    for (int k = 0; k <= 2; ++k) T(c->Bq[l][k]);
  }
  if (c->cf) {
    c->cf_Bl_d = a.get<double>(static_cast<int64_t>(c->cf_Bl_h.size()));
    c->cf_Bl_f = a.get<float>(static_cast<int64_t>(c->cf_Bl_h.size()));
    c->cf_first = a.get<int>(static_cast<int64_t>(c->cf_first_h.size()));
    c->cf_chunks = a.get<int>(static_cast<int64_t>(c->cf_chunks_h.size()));
    c->cf_B2_d = a.get<double>(static_cast<int64_t>(c->cf_B2_h.size()));
    c->qf_win = a.get<double>(static_cast<int64_t>(c->qf_win_h.size()));
    c->qf_wd = a.get<double>(static_cast<int64_t>(c->qf_wd_h.size()));
  }
  T(c->Mt_x); T(c->Wt_x); T(c->Bt0); T(c->Bt1); T(c->BtT); T(c->Gt); T(c->Ut); T(c->UtT);
  c->DEw.d = a.get<double>(static_cast<int64_t>(c->DEw.npad) * c->DEw.npad);
  for (st_iga_ctx::Dense* D : {&c->DUt, &c->DUtT, &c->DUs[0], &c->DUs[1], &c->DUs[2], &c->DUsT[0], &c->DUsT[1],
                               &c->DUsT[2]}) {
    if (D->npad == 0) continue;
    D->d = a.get<double>(static_cast<int64_t>(D->npad) * D->npad);
    D->f = a.get<float>(static_cast<int64_t>(D->npad) * D->npad);
    if (bf) D->b = a.get<bf16>(static_cast<int64_t>(D->npad) * D->npad);
  }
  c->lam_d = a.get<double>(c->Ns);
  c->lam_f = a.get<float>(c->Ns);
  c->mu_d = a.get<double>(c->Nt);
  c->l_d = a.get<double>(c->Nt);
  c->mu_f = a.get<float>(c->Nt);
  c->l_f = a.get<float>(c->Nt);
  c->kind_d = a.get<int>(c->Nt);
  c->el_t_s = a.get<int>(c->nelt);
  c->el_t_c = a.get<int>(c->nelt);
  c->win_t_s = a.get<int>(c->Nt);
  c->win_t_c = a.get<int>(c->Nt);
  for (int l = 0; l < d; ++l) {
    c->el_s_s[l] = a.get<int>(c->nel[l]);
    c->el_s_c[l] = a.get<int>(c->nel[l]);
    c->win_s_s[l] = a.get<int>(c->n[l]);
    c->win_s_c[l] = a.get<int>(c->n[l]);
  }
  if (c->exact_react) {
    const int64_t nq = static_cast<int64_t>(c->dir[d].Q) * c->Qs;
    c->Cq_d = a.get<double>(nq);
    if (mixed) c->Cq_f = a.get<float>(nq);
    c->re0 = a.get<int>(c->nt);
    c->re1 = a.get<int>(c->nt);
    if (c->sc_on) {
      c->Rq_d = a.get<double>(nq);
      if (mixed) c->Rq_f = a.get<float>(nq);
    }
  }
  if (c->supg) {
    for (int l = 0; l < d; ++l) T(c->Ls[l]);
    T(c->Wtau_x);
    T(c->BtTs);
    c->Bts_d = a.get<double>(static_cast<int64_t>(c->Bts_h.size()));
    if (mixed) c->Bts_f = a.get<float>(static_cast<int64_t>(c->Bts_h.size()));
    c->scfac_d = a.get<double>(static_cast<int64_t>(c->scfac_h.size()));
  }
  if (c->banded) {
    const int64_t kw = 2 * c->P.p_t + 1;
    c->bandA_d = a.get<double>(c->Nt * kw);
    c->bandB_d = a.get<double>(c->Nt * kw);
    c->bandF_d = a.get<double>(c->Ns * c->Nt * kw);
    if (mixed) c->bandF_f = a.get<float>(c->Ns * c->Nt * kw);
    c->rowsum_d = a.get<double>(std::max<int64_t>(2LL * c->dir[d].Q, 2LL * c->maxR));
  }
  c->wq_s = a.get<double>(c->Qs);
  c->wq_t = a.get<double>(c->dir[d].Q);
  for (int l = 0; l < d; ++l) c->xq_dev[l] = a.get<double>(c->dir[l].Q);
  c->tq_dev = a.get<double>(c->dir[d].Q);
  const int R2 = 2 * c->maxR;
  const int WB = 2 * c->P.p_t + 1;
  c->Vth = a.get<double>(c->Ns * c->maxR);
  c->Vc = a.get<double>(c->Ns * c->maxR);
  c->Psi = a.get<double>(static_cast<int64_t>(R2) * c->Qs);
  c->NtP = c->Nt + 8;   // row stride of the time tables: 8 zero rows past the last
  c->Tr = a.get<double>(static_cast<int64_t>(R2) * c->NtP * WB);
  c->Tr_f = a.get<float>(static_cast<int64_t>(R2) * c->NtP * WB);
  for (int k = 0; k < 4; ++k) c->t4[k] = a.get<double>(c->nfull);
  for (int k = 0; k < 2; ++k) c->big[k] = a.get<double>(c->big_len);
  c->VT = a.get<double>(static_cast<int64_t>(c->maxR) * c->Ns);
  c->sol_rhs = a.get<double>(c->nunk);
  c->sol_dx = a.get<double>(c->nunk);
  const int m = c->opt.restart;
  const size_t bsz = mixed ? sizeof(float) : sizeof(double);   // Krylov basis storage
  // basis columns padded to 64 elements so every column keeps the alignment
  // of the vectorised kernels
  c->ldb = (c->nunk + 63) & ~static_cast<int64_t>(63);
  c->Vb = a.take(static_cast<size_t>(m + 1) * c->ldb * bsz);
  c->Zb = a.take(static_cast<size_t>(m) * c->ldb * bsz);
  c->rk = a.get<double>(c->nunk);
  c->xk = a.get<double>(c->nunk);
  c->wk = a.get<double>(c->nunk);
  c->dk = a.get<double>(c->nunk);
  c->bk = a.get<double>(c->nunk);
  c->grid = a.get<double>(c->nunk);
  c->grid2 = a.get<double>(c->nunk);
  c->Cg = a.get<double>(c->nunk);
  c->E = a.get<double>(static_cast<int64_t>(c->nelt) * c->Nels);
  c->rfull = a.get<double>(c->nfull);
  c->nb_red = reduce_blocks(c->nfull);
  const int64_t chunk_pts = static_cast<int64_t>(c->chunk_el) * c->nqt * c->Qs;
  const int nchunks = (c->nelt + c->chunk_el - 1) / c->chunk_el;
  c->nb_part = static_cast<int>((chunk_pts + 255) / 256) * nchunks + 1;
  if (c->qf) {
    const int64_t Qin = (d == 3) ? static_cast<int64_t>(c->Q[0]) * c->Q[1] : c->Q[0];
    // blocks of the fused quadrature kernel: column blocks padded to a multiple of 8
    const int64_t nbf = ((Qin + 63) / 64 + 7) / 8 * 8 * c->nelt * c->cf_nchunk + 1;
    c->nb_part = static_cast<int>(std::max<int64_t>(c->nb_part, nbf));
  }
  // reduction partials: up to 2 (m + 1) <= 130 sums per block (two-vector multi-dot)
  c->part = a.get<double>(std::max<int64_t>(static_cast<int64_t>(c->nb_red) * 130, 2 * static_cast<int64_t>(c->nb_part)));
  c->dsc = a.get<double>(1024);
  c->givens = a.get<double>(givens_layout(c->opt.restart).total);
  c->gram_nb = static_cast<int>(std::min<int64_t>(512, (c->Ns + 31) / 32));
  c->gram = a.get<double>(static_cast<int64_t>(c->gram_nb) * c->Nt * c->Nt);
  c->tmpR = a.get<double>(static_cast<int64_t>(c->Nt) * c->maxR + 2 * c->maxR);
  if (mixed) {
    // low-precision operator: FP32 in both mixed modes
    c->Psi_f = a.get<float>(static_cast<int64_t>(R2) * c->Qs);
    for (int k = 0; k < 4; ++k) c->t4f[k] = a.get<float>(c->nfull);
    for (int k = 0; k < 2; ++k) c->bigf[k] = a.get<float>(c->big_len);
    c->xf = a.get<float>(c->nunk);
    c->yf = a.get<float>(c->nunk);
    if (bf) {  // BF16-storage preconditioner
      for (int k = 0; k < 4; ++k) c->t4b[k] = a.get<bf16>(c->nfull);
      c->xb = a.get<bf16>(c->nunk);
      c->yb = a.get<bf16>(c->nunk);
    }
  }
}

template <class X>
void up(const std::vector<X>& h, const X* d, hipStream_t s) {
  if (!h.empty()) CK(hipMemcpyAsync(const_cast<X*>(d), h.data(), h.size() * sizeof(X), hipMemcpyHostToDevice, s));
}

void upload_tab(Tab& t, hipStream_t s, std::vector<std::vector<float>>& keep) {
  if (!t.h.c0.empty()) up(t.h.c0, t.d.c0, s);
  up(t.h.col, t.d.col, s);
  up(t.h.coef, t.d.coef, s);
  keep.emplace_back(t.h.coef.begin(), t.h.coef.end());
  up(keep.back(), t.f.coef, s);
}

void upload_all(st_iga_ctx* c, hipStream_t s) {
  std::vector<std::vector<float>> keepf;
  std::vector<std::vector<int>> keepi;
  std::vector<std::vector<double>> keepd;
  const int d = c->d;
  for (int l = 0; l < d; ++l) {
    for (Tab* t : {&c->Ms[l], &c->Ks[l], &c->BqT[l], &c->Hs[l], &c->Gs[l], &c->Us[l], &c->UsT[l], &c->Bq[l][0],
                   &c->Bq[l][1], &c->Bq[l][2]})
      upload_tab(*t, s, keepf);
  }
  for (Tab* t : {&c->Mt_x, &c->Wt_x, &c->Bt0, &c->Bt1, &c->BtT, &c->Gt, &c->Ut, &c->UtT}) upload_tab(*t, s, keepf);
  if (c->cf) {
    up(c->cf_Bl_h, static_cast<const double*>(c->cf_Bl_d), s);
    keepf.emplace_back(c->cf_Bl_h.begin(), c->cf_Bl_h.end());
    up(keepf.back(), static_cast<const float*>(c->cf_Bl_f), s);
    up(c->cf_first_h, static_cast<const int*>(c->cf_first), s);
    up(c->cf_chunks_h, static_cast<const int*>(c->cf_chunks), s);
    up(c->cf_B2_h, static_cast<const double*>(c->cf_B2_d), s);
    up(c->qf_win_h, static_cast<const double*>(c->qf_win), s);
    up(c->qf_wd_h, static_cast<const double*>(c->qf_wd), s);
  }
  up(c->DEw.h, static_cast<const double*>(c->DEw.d), s);
  for (st_iga_ctx::Dense* D : {&c->DUt, &c->DUtT, &c->DUs[0], &c->DUs[1], &c->DUs[2], &c->DUsT[0], &c->DUsT[1],
                               &c->DUsT[2]}) {
    if (D->npad == 0) continue;
    up(D->h, static_cast<const double*>(D->d), s);
    keepf.emplace_back(D->h.begin(), D->h.end());
    up(keepf.back(), static_cast<const float*>(D->f), s);
    if (D->b) convert<float, bf16>(D->f, D->b, static_cast<int64_t>(D->npad) * D->npad, s);
  }
  up(c->lam_s_h, static_cast<const double*>(c->lam_d), s);
  keepf.emplace_back(c->lam_s_h.begin(), c->lam_s_h.end());
  up(keepf.back(), static_cast<const float*>(c->lam_f), s);
  std::vector<double> mu(c->Nt, 0.0), l(c->Nt, 0.0);
  std::vector<int> kind(c->Nt, 2);
  for (int i = 0; i < c->Nt - 1; ++i) { mu[i] = c->fd.mu[i]; l[i] = c->fd.l[i]; kind[i] = c->fd.kind[i]; }
  keepd.push_back(mu); up(keepd.back(), static_cast<const double*>(c->mu_d), s);
  keepd.push_back(l); up(keepd.back(), static_cast<const double*>(c->l_d), s);
  keepf.emplace_back(mu.begin(), mu.end()); up(keepf.back(), static_cast<const float*>(c->mu_f), s);
  keepf.emplace_back(l.begin(), l.end()); up(keepf.back(), static_cast<const float*>(c->l_f), s);
  keepi.push_back(kind); up(keepi.back(), static_cast<const int*>(c->kind_d), s);
  // element ranges (Gauss points of each element) and support-extension windows
  const Dir1D& T = c->dir[d];
  {
    std::vector<int> st(c->nelt), ct(c->nelt, T.nq);
    for (int e = 0; e < c->nelt; ++e) st[e] = e * T.nq;
    keepi.push_back(st); up(keepi.back(), static_cast<const int*>(c->el_t_s), s);
    keepi.push_back(ct); up(keepi.back(), static_cast<const int*>(c->el_t_c), s);
    std::vector<int> e0, e1;
    support_windows(T, 1, e0, e1);
    std::vector<int> cnt(e0.size());
    for (size_t i = 0; i < e0.size(); ++i) cnt[i] = e1[i] - e0[i];
    keepi.push_back(e0); up(keepi.back(), static_cast<const int*>(c->win_t_s), s);
    keepi.push_back(cnt); up(keepi.back(), static_cast<const int*>(c->win_t_c), s);
  }
  for (int l2 = 0; l2 < d; ++l2) {
    const Dir1D& D = c->dir[l2];
    std::vector<int> st(D.nel), ct(D.nel, D.nq);
    for (int e = 0; e < D.nel; ++e) st[e] = e * D.nq;
    keepi.push_back(st); up(keepi.back(), static_cast<const int*>(c->el_s_s[l2]), s);
    keepi.push_back(ct); up(keepi.back(), static_cast<const int*>(c->el_s_c[l2]), s);
    std::vector<int> e0, e1;
    support_windows(D, 0, e0, e1);
    std::vector<int> cnt(e0.size());
    for (size_t i = 0; i < e0.size(); ++i) cnt[i] = e1[i] - e0[i];
    keepi.push_back(e0); up(keepi.back(), static_cast<const int*>(c->win_s_s[l2]), s);
    keepi.push_back(cnt); up(keepi.back(), static_cast<const int*>(c->win_s_c[l2]), s);
  }
  // tensor spatial weights and time weights
  std::vector<double> ws(c->Qs, 1.0);
  for (int64_t q = 0; q < c->Qs; ++q) {
    int64_t r = q;
    double w = 1.0;
    for (int l2 = 0; l2 < d; ++l2) {
      w *= c->dir[l2].wq[r % c->Q[l2]];
      r /= c->Q[l2];
    }
    ws[q] = w;
  }
  keepd.push_back(ws); up(keepd.back(), static_cast<const double*>(c->wq_s), s);
  up(T.wq, static_cast<const double*>(c->wq_t), s);
  for (int l = 0; l < d; ++l) up(c->dir[l].xq, static_cast<const double*>(c->xq_dev[l]), s);
  up(T.xq, static_cast<const double*>(c->tq_dev), s);
  if (c->exact_react) {
    up(c->re0_h, static_cast<const int*>(c->re0), s);
    up(c->re1_h, static_cast<const int*>(c->re1), s);
  }
  if (c->supg) {
    for (int l = 0; l < d; ++l) upload_tab(c->Ls[l], s, keepf);
    upload_tab(c->Wtau_x, s, keepf);
    upload_tab(c->BtTs, s, keepf);
    up(c->Bts_h, static_cast<const double*>(c->Bts_d), s);
    if (c->Bts_f) {
      keepf.emplace_back(c->Bts_h.begin(), c->Bts_h.end());
      up(keepf.back(), static_cast<const float*>(c->Bts_f), s);
    }
    up(c->scfac_h, static_cast<const double*>(c->scfac_d), s);
  }
  if (c->banded) up(c->band_B_h, static_cast<const double*>(c->bandB_d), s);
  CK(hipStreamSynchronize(s));
}

// Factorize the per-mode time matrices T_j = A + lam_j B of the banded
// preconditioner, lam_j the spatial eigenvalue sums without the reaction
// shift, B = M_t (+ W_tau with SUPG) and
//   A = C_m W_t + int max(cr, a c1) b_j b_i + sum_k int max(C_m tau_k th, 0) b_j^(k) b_i^(k)   (Galerkin / SU)
//   A = C_m (W_t + K_t^tau) + int cr b_j (b_i + tau b_i') + int sc b_j' b_i'  (SUPG + SC)
// with the time profiles cr (reaction coefficient, clipped at 0), th (theta)
// and sc (shock capturing) at the time Gauss points (empty: zero).
void time_factor(st_iga_ctx* c, hipStream_t s) {
  const Dir1D& T = c->dir[c->d];
  const int pt = c->P.p_t, nt = c->nt;
  auto prof = [&](const std::vector<double>& v, int q) { return v.empty() ? 0.0 : std::max(v[q], 0.0); };
  // the factorization has no pivoting: its symmetric part must stay positive
  // definite.  SUPG's tau K_t term ensures that; otherwise the reaction
  // profile is floored at the shift a c1 of the fast diagonalization (> 0,
  // checked at setup) and the theta terms at 0
  const double floor_cr = c->supg ? 0.0 : c->P.a * c->P.c1;
  std::vector<double> crt(T.Q);
  for (int q = 0; q < T.Q; ++q) crt[q] = std::max(prof(c->prof_cr, q), floor_cr);
  std::vector<double> A = c->timeA0_full;
  auto add = [&](const std::vector<double>& G) {
    for (size_t k = 0; k < A.size(); ++k) A[k] += G[k];
  };
  add(gram1d(T, 0, 0, &crt));
  if (c->supg) {
    std::vector<double> crtau(T.Q), sct(T.Q);
    for (int q = 0; q < T.Q; ++q) {
      crtau[q] = crt[q] * c->tq_h[q];
      sct[q] = prof(c->prof_sc, q);
    }
    add(gram1d(T, 1, 0, &crtau));
    add(gram1d(T, 1, 1, &sct));
  } else if (c->opt.su == 1 && !c->prof_th.empty()) {
    for (int k = 1; k <= pt; ++k) {
      std::vector<double> wk(T.Q);
      for (int q = 0; q < T.Q; ++q)
        wk[q] = std::max(c->P.Cm * c->tauq[static_cast<size_t>(k - 1) * T.Q + q] * prof(c->prof_th, q), 0.0);
      add(gram1d(T, k, k, &wk));
    }
  }
  const std::vector<double> band = band_rows(A, nt, pt);
  CK(hipMemcpyAsync(c->bandA_d, band.data(), band.size() * sizeof(double), hipMemcpyHostToDevice, s));
  if (!band_factor(c->bandA_d, c->bandB_d, c->Nt, c->lam_d, c->P.a * c->P.c1, c->Ns, pt, c->bandF_d, s))
    throw Fail{ST_IGA_EINVAL, "banded preconditioner: time degree above 5"};
  const int64_t nf = c->Ns * c->Nt * (2 * pt + 1);
  if (c->bandF_f) convert<double, float>(c->bandF_d, c->bandF_f, nf, s);
  // the host vectors above are released on return: wait for the upload
  CK(hipStreamSynchronize(s));
  check_launch();
}

// Total Gauss weight of the spatial domain (its measure).
double space_volume(const st_iga_ctx* c) {
  double vol = 1.0;
  for (int l = 0; l < c->d; ++l) {
    double sw = 0.0;
    for (double w : c->dir[l].wq) sw += w;
    vol *= sw;
  }
  return vol;
}

// ------------------------------------------------------------------ operators
template <class S, class C>
struct Ops {
  // per-precision accessors
  static const DTable<C>& tab(const Tab& t);
};
template <>
const DTable<double>& Ops<double, double>::tab(const Tab& t) { return t.d; }
template <>
const DTable<float>& Ops<float, float>::tab(const Tab& t) { return t.f; }
template <>
const DTable<float>& Ops<bf16, float>::tab(const Tab& t) { return t.f; }

template <class S>
struct Bufs {
  S* t4[4];
  S* big[2];
  const S* Psi;
};

// Apply the tensor chain along spatial axes: x has layout [L][m_d]..[m_1] with
// m_l = in dims; apply tabs[l] along axis l (output dims out[l]); ping-pong
// between bufA/bufB; the last step writes to `dst` with (alpha, beta).  Axes
// are taken x_1 first when the chain grows the array (expansion to Gauss
// points) and x_d first when it shrinks it, so the fastest-axis step always
// works on the smallest array.
template <class S, class C>
const S* spatial_chain(st_iga_ctx* c, const Tab* const* tabs, const S* x, int64_t L, const int* in_dims,
                       const int* out_dims, S* bufA, S* bufB, S* dst, C alpha, C beta, hipStream_t s) {
  const int d = c->d;
  int dims[3];
  int64_t grow = 0;
  for (int l = 0; l < d; ++l) {
    dims[l] = in_dims[l];
    grow += out_dims[l] - in_dims[l];
  }
  const S* cur = x;
  S* bufs[2] = {bufA, bufB};
  int pb = 0;
  for (int step = 0; step < d; ++step) {
    const int l = grow >= 0 ? step : d - 1 - step;
    int64_t inner = 1, outer = L;
    for (int k = 0; k < l; ++k) inner *= dims[k];
    for (int k = l + 1; k < d; ++k) outer *= dims[k];
    const bool last = (step == d - 1);
    S* out = last ? dst : bufs[pb];
    gather<S, S, C>(Ops<S, C>::tab(*tabs[l]), cur, out, outer, inner, dims[l], 0, last ? alpha : C(1), last ? beta : C(0), s);
    dims[l] = out_dims[l];
    cur = out;
    pb ^= 1;
  }
  return cur;
}

// y (N_t layers) = A_lin x (+ reaction terms when with_react), x with L layers
// (L = N_t, in_base 1: unknowns; L = n_t, in_base 0: full vectors).
template <class S, class C>
void apply_impl(st_iga_ctx* c, const S* x, S* y, int L, int in_base, bool with_su, bool with_react, Bufs<S>& B,
                hipStream_t s) {
  const int d = c->d;
  const st_iga_problem& P = c->P;
  const int64_t Ns = c->Ns;
  S *a = B.t4[0], *b = B.t4[1], *e = B.t4[2], *f = B.t4[3];
  const int nn[3] = {c->n[0], c->n[1], c->n[2]};
  // spatial constant part: SM = (M_d..M_1) x, SK = K_s x
  S* SM;
  S* SK;
  kprof_gather_class(K_BANDED);
  if (d == 1) {
    gather<S, S, C>(Ops<S, C>::tab(c->Ms[0]), x, a, L, 1, nn[0], 0, C(1), C(0), s);
    gather<S, S, C>(Ops<S, C>::tab(c->Ks[0]), x, b, L, 1, nn[0], 0, C(P.sigma[0]), C(0), s);
    SM = a;
    SK = b;
  } else {
    // axis l >= 1: (M_l a, sigma_l K_l a + s M_l b) in one dual sweep when
    // the two tables share their windows, else three gathers
    auto axis = [&](int l, const S* xa, const S* xb, S* oa, S* ob, int64_t outer, int64_t inner, C sb) {
      if (c->dual[l] && gather_dual<S, C>(Ops<S, C>::tab(c->Ms[l]), Ops<S, C>::tab(c->Ks[l]), xa, xb, oa, ob, outer,
                                          inner, nn[l], 0, C(P.sigma[l]), sb, s))
        return;
      gather<S, S, C>(Ops<S, C>::tab(c->Ms[l]), xa, oa, outer, inner, nn[l], 0, C(1), C(0), s);
      gather<S, S, C>(Ops<S, C>::tab(c->Ks[l]), xa, ob, outer, inner, nn[l], 0, C(P.sigma[l]), C(0), s);
      gather<S, S, C>(Ops<S, C>::tab(c->Ms[l]), xb, ob, outer, inner, nn[l], 0, sb, C(1), s);
    };
    if (d == 2) {
      gather<S, S, C>(Ops<S, C>::tab(c->Ms[0]), x, a, L * nn[1], 1, nn[0], 0, C(1), C(0), s);
      gather<S, S, C>(Ops<S, C>::tab(c->Ks[0]), x, b, L * nn[1], 1, nn[0], 0, C(1), C(0), s);
      axis(1, a, b, e, f, L, nn[0], C(P.sigma[0]));
      SM = e;
      SK = f;
    } else {
      gather<S, S, C>(Ops<S, C>::tab(c->Ms[0]), x, a, L * nn[1] * nn[2], 1, nn[0], 0, C(1), C(0), s);
      gather<S, S, C>(Ops<S, C>::tab(c->Ks[0]), x, b, L * nn[1] * nn[2], 1, nn[0], 0, C(1), C(0), s);
      axis(1, a, b, e, f, L * nn[2], nn[0], C(P.sigma[0]));     // M2 M1 x, sigma2 M1 K2 x + sigma1 K1 M2 x
      axis(2, e, f, a, b, L, static_cast<int64_t>(nn[0]) * nn[1], C(1));
      SM = a;
      SK = b;
    }
  }
  // time: y = Cm W_t SM + M_t SK (rows X_t, columns per in_base)
  if (!(c->dual[d] && gather_dual<S, C>(Ops<S, C>::tab(c->Mt_x), Ops<S, C>::tab(c->Wt_x), SM, SK, nullptr, y, 1, Ns,
                                        L, in_base, C(P.Cm), C(1), s))) {
    gather<S, S, C>(Ops<S, C>::tab(c->Wt_x), SM, y, 1, Ns, L, in_base, C(P.Cm), C(0), s);
    gather<S, S, C>(Ops<S, C>::tab(c->Mt_x), SK, y, 1, Ns, L, in_base, C(1), C(1), s);
  }
  if (c->supg) {
    // strong-form diffusion of the SUPG term (Section 4.2.2):
    // y -= W_tau (x) sum_l sigma_l (M_d .. L_l .. M_1) x, L_l = int B_j'' B_i
    auto axisL = [&](int l, const S* xa, const S* xb, S* oa, S* ob, int64_t outer, int64_t inner, C sb) {
      if (c->dualL[l] && gather_dual<S, C>(Ops<S, C>::tab(c->Ms[l]), Ops<S, C>::tab(c->Ls[l]), xa, xb, oa, ob, outer,
                                           inner, nn[l], 0, C(P.sigma[l]), sb, s))
        return;
      if (oa) gather<S, S, C>(Ops<S, C>::tab(c->Ms[l]), xa, oa, outer, inner, nn[l], 0, C(1), C(0), s);
      gather<S, S, C>(Ops<S, C>::tab(c->Ls[l]), xa, ob, outer, inner, nn[l], 0, C(P.sigma[l]), C(0), s);
      gather<S, S, C>(Ops<S, C>::tab(c->Ms[l]), xb, ob, outer, inner, nn[l], 0, sb, C(1), s);
    };
    S* SG;
    kprof_gather_class(K_BANDED);
    if (d == 1) {
      gather<S, S, C>(Ops<S, C>::tab(c->Ls[0]), x, a, L, 1, nn[0], 0, C(P.sigma[0]), C(0), s);
      SG = a;
    } else if (d == 2) {
      gather<S, S, C>(Ops<S, C>::tab(c->Ms[0]), x, a, L * nn[1], 1, nn[0], 0, C(1), C(0), s);
      gather<S, S, C>(Ops<S, C>::tab(c->Ls[0]), x, b, L * nn[1], 1, nn[0], 0, C(1), C(0), s);
      axisL(1, a, b, nullptr, e, L, nn[0], C(P.sigma[0]));   // sigma2 L2 M1 x + sigma1 M2 L1 x
      SG = e;
    } else {
      gather<S, S, C>(Ops<S, C>::tab(c->Ms[0]), x, a, L * nn[1] * nn[2], 1, nn[0], 0, C(1), C(0), s);
      gather<S, S, C>(Ops<S, C>::tab(c->Ls[0]), x, b, L * nn[1] * nn[2], 1, nn[0], 0, C(1), C(0), s);
      axisL(1, a, b, e, f, L * nn[2], nn[0], C(P.sigma[0]));
      axisL(2, e, f, nullptr, a, L, static_cast<int64_t>(nn[0]) * nn[1], C(1));
      SG = a;
    }
    gather<S, S, C>(Ops<S, C>::tab(c->Wtau_x), SG, y, 1, Ns, L, in_base, C(-1), C(1), s);
  }
  // low-rank coefficient terms
  const int r0 = with_su ? 0 : c->Rth;
  const int r1 = with_react ? c->Rth + c->Rc : c->Rth;
  // M_R with C_r at every Gauss point, and the shock-capturing term
  const bool pw_react = with_react && c->exact_react;
  const bool pw_sc = with_su && c->sc_on;
  const bool pointwise = pw_react || pw_sc;
  kprof_gather_class(K_EXPAND);
  struct Reset { ~Reset() { kprof_gather_class(K_GATHER); } } reset_cls;
  if (r1 <= r0 && !pointwise) return;
  const Tab* ex[3] = {&c->Bq[0][0], &c->Bq[1][0], &c->Bq[2][0]};
  const Tab* pr[3] = {&c->BqT[0], &c->BqT[1], &c->BqT[2]};
  const int qd[3] = {c->Q[0], c->Q[1], c->Q[2]};
  S* Z = B.big[0];
  S* W2 = B.big[1];
  S* bufA = (d == 3) ? Z : W2;   // intermediates never alias the step that reads them
  S* bufB = W2;
  const C* Tr = std::is_same<C, double>::value ? reinterpret_cast<const C*>(c->Tr) : reinterpret_cast<const C*>(c->Tr_f);
  const int p = P.p_t;
  if (c->cf && !pointwise) {
    // expand along the faster axes, then one fused kernel along the slowest
    const C* Bl = std::is_same<C, double>::value ? reinterpret_cast<const C*>(c->cf_Bl_d)
                                                 : reinterpret_cast<const C*>(c->cf_Bl_f);
    const int nd = nn[d - 1];
    const int64_t Qin = (d == 3) ? static_cast<int64_t>(qd[0]) * qd[1] : qd[0];
    for (int t0 = 0; t0 < c->Nt; t0 += c->cf_slab) {
      const int t1 = std::min(c->Nt, t0 + c->cf_slab);
      const int lo = std::max(0, t0 + 1 - p - in_base);
      const int hi = std::min(L - 1, t1 + p - in_base);
      const int nl = hi - lo + 1;
      const int rows = t1 - t0;
      const S* xs = x + static_cast<int64_t>(lo) * Ns;
      S* ys = y + static_cast<int64_t>(t0) * Ns;
      S* X1 = B.big[0];
      S* Y2 = B.big[1];
      if (d == 2) {
        gather<S, S, C>(Ops<S, C>::tab(*ex[0]), xs, X1, static_cast<int64_t>(nl) * nn[1], 1, nn[0], 0, C(1), C(0), s);
        coef_fused<S, C>(Tr, B.Psi, r0, r1, c->NtP, t0, t1, p, P.p_s, X1, nl, in_base + lo, Bl, c->cf_first,
                         c->cf_chunks, c->cf_nchunk, nd, Qin, Y2, c->Qs, s);
        gather<S, S, C>(Ops<S, C>::tab(*pr[0]), Y2, ys, static_cast<int64_t>(rows) * nn[1], 1, qd[0], 0, C(1), C(1), s);
      } else {
        S* X2 = X1 + static_cast<int64_t>(nl) * nn[2] * nn[1] * qd[0];
        S* Y1 = Y2 + static_cast<int64_t>(rows) * nn[2] * Qin;
        gather<S, S, C>(Ops<S, C>::tab(*ex[0]), xs, X1, static_cast<int64_t>(nl) * nn[2] * nn[1], 1, nn[0], 0, C(1),
                        C(0), s);
        gather<S, S, C>(Ops<S, C>::tab(*ex[1]), X1, X2, static_cast<int64_t>(nl) * nn[2], qd[0], nn[1], 0, C(1), C(0),
                        s);
        coef_fused<S, C>(Tr, B.Psi, r0, r1, c->NtP, t0, t1, p, P.p_s, X2, nl, in_base + lo, Bl, c->cf_first,
                         c->cf_chunks, c->cf_nchunk, nd, Qin, Y2, c->Qs, s);
        gather<S, S, C>(Ops<S, C>::tab(*pr[1]), Y2, Y1, static_cast<int64_t>(rows) * nn[2], qd[0], qd[1], 0, C(1), C(0),
                        s);
        gather<S, S, C>(Ops<S, C>::tab(*pr[0]), Y1, ys, static_cast<int64_t>(rows) * nn[2] * nn[1], 1, qd[0], 0, C(1),
                        C(1), s);
      }
    }
    return;
  }
  // slabs of output time rows; each expands only the input layers its time window reads
  for (int t0 = 0; t0 < c->Nt; t0 += c->slab) {
    const int t1 = std::min(c->Nt, t0 + c->slab);
    const int lo = std::max(0, t0 + 1 - p - in_base);
    const int hi = std::min(L - 1, t1 + p - in_base);
    const int nl = hi - lo + 1;
    const S* xs = x + static_cast<int64_t>(lo) * Ns;
    if (d == 1) gather<S, S, C>(Ops<S, C>::tab(*ex[0]), xs, Z, nl, 1, nn[0], 0, C(1), C(0), s);
    else spatial_chain<S, C>(c, ex, xs, nl, nn, qd, bufA, bufB, Z, C(1), C(0), s);
    if (r1 > r0) time_mix<S, C>(Tr, B.Psi, r0, r1, c->NtP, t0, t1, p, Z, nl, in_base + lo, W2, c->Qs, s);
    if (pointwise) {
      const bool dbl = std::is_same<C, double>::value;
      const C* Cq = !pw_react ? nullptr
                              : dbl ? reinterpret_cast<const C*>(c->Cq_d) : reinterpret_cast<const C*>(c->Cq_f);
      const C* Rq = !pw_sc ? nullptr
                           : dbl ? reinterpret_cast<const C*>(c->Rq_d) : reinterpret_cast<const C*>(c->Rq_f);
      const C* Bv = !c->supg ? nullptr
                             : dbl ? reinterpret_cast<const C*>(c->Bts_d) : reinterpret_cast<const C*>(c->Bts_f);
      react_point<S, C>(Z, nl, in_base + lo, Ops<S, C>::tab(c->Bt0), Bv, Ops<S, C>::tab(c->Bt1).coef, c->re0, c->re1,
                        Cq, Rq, c->Qs, t0, t1, p, W2, r1 > r0 ? C(1) : C(0), s);
    }
    S* ys = y + static_cast<int64_t>(t0) * Ns;
    if (d == 1) gather<S, S, C>(Ops<S, C>::tab(*pr[0]), W2, ys, t1 - t0, 1, qd[0], 0, C(1), C(1), s);
    else spatial_chain<S, C>(c, pr, W2, t1 - t0, qd, nn, Z, (d == 3 ? W2 : Z), ys, C(1), C(1), s);
  }
}

// The time-mix kernel indexes inputs by full time index minus in_base; for
// unknown vectors (layer k = full index k+1) in_base = 1, for full vectors 0.

template <class C>
const C* dmat(const st_iga_ctx::Dense& D);
template <>
const double* dmat<double>(const st_iga_ctx::Dense& D) { return D.d; }
template <>
const float* dmat<float>(const st_iga_ctx::Dense& D) { return D.f; }

// Dense matrices along every spatial axis: x [L][n_d..n_1] -> dst; intermediates alternate bufA/bufB.
template <class S, class C>
void dense_spatial(st_iga_ctx* c, const st_iga_ctx::Dense* const* M, const S* x, int64_t L, S* bufA, S* bufB, S* dst,
                   hipStream_t s) {
  const int d = c->d;
  const S* cur = x;
  S* bufs[2] = {bufA, bufB};
  int pb = 0;
  for (int l = 0; l < d; ++l) {
    int64_t inner = 1, outer = L;
    for (int k = 0; k < l; ++k) inner *= c->n[k];
    for (int k = l + 1; k < d; ++k) outer *= c->n[k];
    S* out = (l == d - 1) ? dst : bufs[pb];
    bool done = false;
    if constexpr (std::is_same<S, bf16>::value)
      done = M[l]->b && dense_mode_b16(M[l]->b, M[l]->n, M[l]->npad, cur, out, outer, inner, s);
    if (!done) dense_mode<S, C>(dmat<C>(*M[l]), M[l]->n, M[l]->npad, cur, out, outer, inner, s);
    cur = out;
    pb ^= 1;
  }
}

template <class S, class C>
void precond_impl(st_iga_ctx* c, const S* r, S* z, Bufs<S>& B, hipStream_t s) {
  const int64_t Ns = c->Ns;
  const int Nt = c->Nt;
  const st_iga_ctx::Dense* UT[3] = {&c->DUsT[0], &c->DUsT[1], &c->DUsT[2]};
  const st_iga_ctx::Dense* U[3] = {&c->DUs[0], &c->DUs[1], &c->DUs[2]};
  S *a = B.t4[0], *b = B.t4[1], *e = B.t4[2];
  // spatial forward transforms: a = (U_d^T .. U_1^T) r
  dense_spatial<S, C>(c, UT, r, Nt, b, e, a, s);
  const C* lam = std::is_same<C, double>::value ? reinterpret_cast<const C*>(c->lam_d) : reinterpret_cast<const C*>(c->lam_f);
  const C* mu = std::is_same<C, double>::value ? reinterpret_cast<const C*>(c->mu_d) : reinterpret_cast<const C*>(c->mu_f);
  const C* l = std::is_same<C, double>::value ? reinterpret_cast<const C*>(c->l_d) : reinterpret_cast<const C*>(c->l_f);
  if (c->banded) {
    // exact banded solve per spatial mode in time
    const C* F = std::is_same<C, double>::value ? reinterpret_cast<const C*>(c->bandF_d)
                                                : reinterpret_cast<const C*>(c->bandF_f);
    if (!band_solve<S, C>(F, Nt, Ns, c->P.p_t, a, b, s)) throw Fail{ST_IGA_EINVAL, "time degree above 5"};
    dense_spatial<S, C>(c, U, b, Nt, a, e, z, s);
    return;
  }
  bool fused = false;
  if constexpr (std::is_same<C, float>::value) {
    // FP32: time transforms and arrowhead in one pass, b = U_t core^{-1} U_t^T a
    fused = c->DUtT.npad == c->DUt.npad &&
            time_core<S>(dmat<C>(c->DUtT), dmat<C>(c->DUt), Nt, c->DUtT.npad, a, b, Ns, lam, mu, c->fd_np, l,
                         static_cast<float>(c->fd.sigma), static_cast<float>(c->P.Cm), s);
  }
  if (!fused) {
    // time forward: b = U_t^T a
    dense_mode<S, C>(dmat<C>(c->DUtT), Nt, c->DUtT.npad, a, b, 1, Ns, s);
    // arrowhead core
    arrowhead<S, C>(b, a, lam, mu, c->fd_np, l, C(c->fd.sigma), C(c->P.Cm), Nt, Ns, s);
    // time backward: b = U_t a
    dense_mode<S, C>(dmat<C>(c->DUt), Nt, c->DUt.npad, a, b, 1, Ns, s);
  }
  // spatial backward: z = (U_d .. U_1) b
  dense_spatial<S, C>(c, U, b, Nt, a, e, z, s);
}

Bufs<double> bufs64(st_iga_ctx* c) {
  Bufs<double> B;
  for (int k = 0; k < 4; ++k) B.t4[k] = c->t4[k];
  B.big[0] = c->big[0];
  B.big[1] = c->big[1];
  B.Psi = c->Psi;
  return B;
}

// ------------------------------------------------------------------ reductions
double dev_norm(st_iga_ctx* c, const double* x, int64_t n, hipStream_t s) {
  const int nb = reduce_blocks(n);
  sumsq_partial(x, n, c->part, nb, s);
  finalize_sum(c->part, nb, 1, c->dsc + 900, s);
  double h;
  CK(hipMemcpyAsync(&h, c->dsc + 900, sizeof(double), hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  return std::sqrt(h);
}

double dev_absmax(st_iga_ctx* c, const double* x, int64_t n, hipStream_t s) {
  const int nb = reduce_blocks(n);
  absmax_partial(x, n, c->part, nb, s);
  finalize_max(c->part, nb, c->dsc + 901, s);
  double h;
  CK(hipMemcpyAsync(&h, c->dsc + 901, sizeof(double), hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  return h;
}

// Stagnation of a restarted iteration: a cycle (FGMRES restart or refinement
// step) whose true residual falls by less than the relative amount
// stall_reduction counts as a stall; stall_cycles stalls in a row end the
// solve with ENOCONV (stall_cycles = 0: never).
struct Stall {
  st_iga_ctx* c;
  double prev;
  const char* what;
  int count = 0;
  Stall(st_iga_ctx* cc, double start, const char* w) : c(cc), prev(start), what(w) {}
  void cycle(double rn) {
    if (c->opt.stall_cycles <= 0) return;
    if (rn > (1.0 - c->opt.stall_reduction) * prev) {
      if (++count >= c->opt.stall_cycles) throw Fail{ST_IGA_ENOCONV, what};
    } else {
      count = 0;
    }
    prev = rn;
  }
};

using Op = std::function<void(const double*, double*)>;
template <class T>
using OpT = std::function<void(const T*, T*)>;

// Right-preconditioned FGMRES(m) on A x = b from x = 0.  The Krylov basis V
// (m+1 vectors) and Z (m vectors) are stored in T (FP64, or FP32 for the inner
// solves of mixed precision); Arnoldi dot products, the Gram-Schmidt updates
// (classical, twice) and the Givens rotations are carried out in FP64.  b, x
// and the restart residual are FP64.  Returns the iteration count; *est is the
// relative residual of the last restart check, computed with the same A.
// Replays fn(stream) from the HIP graph cached for basis column j (captured
// on the library's capture stream on first use, re-captured when the ranks
// changed), or runs it eagerly on s when graphs are off or the per-launch
// profiler is on.
void run_step(st_iga_ctx* c, std::vector<st_iga_ctx::StepGraph>& gv, int j, int m,
              const std::function<void(hipStream_t)>& fn, hipStream_t s) {
  if (c->opt.graphs == 0 || kprof_enabled()) {
    fn(s);
    return;
  }
  if (gv.size() < static_cast<size_t>(m)) gv.resize(m);
  auto& g = gv[j];
  if (g.exec && (g.rth != c->Rth || g.rc != c->Rc)) {
    CK(hipGraphExecDestroy(g.exec));
    g.exec = nullptr;
  }
  if (!g.exec) {
    if (!c->cap_stream) CK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    const hipStream_t cs = c->cap_stream;
    hipGraph_t graph = nullptr;
    CK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    try {
      fn(cs);
    } catch (...) {
      c->op_stream = s;
      hipStreamEndCapture(cs, &graph);
      if (graph) hipGraphDestroy(graph);
      throw;
    }
    CK(hipStreamEndCapture(cs, &graph));
    const hipError_t ie = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      g.exec = nullptr;
      throw Fail{ST_IGA_EDEVICE, std::string("graph instantiation: ") + hipGetErrorString(ie)};
    }
    g.rth = c->Rth;
    g.rc = c->Rc;
  }
  CK(hipGraphLaunch(g.exec, s));
}

// FGMRES(m) as below with the second classical Gram-Schmidt pass of each
// basis vector delayed into the next Arnoldi step (one multi-dot over V for
// both the new vector w and the previous vector u, one fused update): per
// step the basis is read twice instead of four times.  Step j orthogonalizes
// u = column j against columns < j (coefficients s, norm alpha), which
// completes Hessenberg column j - 1 (u is stored divided by alpha_{j-1}:
// entries += alpha_{j-1} s, subdiagonal alpha_{j-1} alpha), and projects w
// on the finished columns <= j.  The last column of a cycle keeps its
// once-orthogonalized subdiagonal (the norm of the projected w).  u is
// neither normalized nor twice orthogonalized when the preconditioner is
// applied to it; flexible GMRES only needs the pairs (z_j, A z_j) that the
// Hessenberg matrix describes.
template <class T>
int fgmres_delayed(st_iga_ctx* c, const OpT<T>& A, const OpT<T>& Pc, const double* b, double* x, double rtol,
                   int maxit, double bnorm, double* est, T* V, T* Z, T* xt, T* yt, hipStream_t s) {
  const int64_t n = c->nunk, ld = c->ldb;
  const int m = c->opt.restart;
  const int nb = reduce_blocks(n);
  fill(x, 0.0, n, s);
  int it = 0;
  double rn = bnorm;
  Stall stall(c, bnorm, "FGMRES stagnated");
  CK(hipMemcpyAsync(c->rk, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  // the Hessenberg matrix, its Givens rotations and the back substitution
  // live on the device (norm_givens, givens_solve); per step the host
  // reads 8 values to decide whether the cycle goes on
  const GivensLayout GL = givens_layout(m);
  double* G = c->givens;
  constexpr int HS = 264;   // pinned slot per step parity
  if (!c->step_host) CK(hipHostMalloc(reinterpret_cast<void**>(&c->step_host), 2 * HS * sizeof(double), 0));
  for (auto& ev : c->step_ev)
    if (!ev) CK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  auto& gv = c->graphs[(std::is_same<T, double>::value ? 0 : 1) + 2];
  // steps alternate between two scalar regions of dsc and of the pinned
  // buffer, so step j + 1 can run while the host reads step j
  auto region = [&](int j) { return c->dsc + (j & 1) * 640; };
  const bool overlap = c->opt.graphs != 0 && !kprof_enabled();
  while (it < maxit) {
    scale_to<T>(c->rk, 1.0 / rn, V, n, s);
    // Hr = 0, g = 0, gpre = (rn, 0, ...)
    fill(G + GL.Hr, 0.0, GL.R - GL.Hr, s);
    fill(G + GL.g, 0.0, GL.ap - GL.g, s);
    fill(G + GL.gpre, rn, 1, s);
    int ncol = 0;
    bool final_col_provisional = true;   // false: the cycle stopped right after completing a column
    // step j on the stream, followed by the copy of its scalars and its event
    auto launch = [&](int j) {
      T* Vj = V + static_cast<int64_t>(j) * ld;
      T* Zj = Z + static_cast<int64_t>(j) * ld;
      T* w = V + static_cast<int64_t>(j + 1) * ld;
      double* D = region(j);
      auto body = [&](hipStream_t ss) {
        c->op_stream = ss;
        Pc(Vj, Zj);
        A(Zj, w);
        c->op_stream = s;
        multidot2_partial<T>(V, ld, j + 1, Vj, w, n, c->part, nb, ss);
        finalize_sum(c->part, nb, 2 * (j + 1), D, ss);
        dcgs_update_partial<T>(V, ld, j, D, n, c->part, nb, D + 128, ss);
        norm_givens(c->part, nb, D, G, GL, m, j, ss);
        // the step's decision values to pinned host memory, inside the
        // replayed graph (one runtime call less per Krylov iteration)
        CK(hipMemcpyAsync(c->step_host + (j & 1) * HS, G + GL.out + (j & 1) * 8, 8 * sizeof(double),
                          hipMemcpyDeviceToHost, ss));
      };
      run_step(c, gv, j, m, body, s);
      CK(hipEventRecord(c->step_ev[j & 1], s));
    };
    int queued = -1;          // last step already on the stream
    double res_prev = -1.0;   // residual estimate one step earlier
    double res_next = rn;     // |g[j]| as left by step j - 1 (the provisional rotation)
    for (int j = 0; j < m && it < maxit; ++j) {
      if (queued < j) launch(j);
      queued = j;
      // step j + 1 needs only device data: queue it before reading step j
      // while the residual estimate is far from the tolerance (a step that
      // turns out unneeded writes only basis columns, the provisional column
      // of R and g entries that the back substitution does not read)
      const double res = std::fabs(res_next);
      const double q = res_prev > 0.0 ? std::min(1.0, res / res_prev) : 0.0;
      if (overlap && j + 1 < m && it + 1 < maxit &&
          (c->opt.graphs == 2 || res * (j == 0 ? 1.0 / 64 : q) > 4.0 * rtol * bnorm)) {
        launch(j + 1);
        queued = j + 1;
      }
      res_prev = res;
      CK(hipEventSynchronize(c->step_ev[j & 1]));
      check_launch();
      const double* hb = c->step_host + (j & 1) * HS;
      ++it;
      // hb: alpha, h, beta, g[j] after completing column j - 1, g[j + 1]
      // after the provisional rotation of column j, flag
      if (hb[5] == 1.0) throw Fail{ST_IGA_ENOCONV, "non-finite Arnoldi coefficients"};
      if (hb[5] == 2.0) throw Fail{ST_IGA_ENOCONV, "zero Krylov start vector"};
      const double alpha = hb[0], beta = hb[2];
      if (j > 0) {
        ncol = j;
        if (alpha == 0.0 || std::fabs(hb[3]) <= rtol * bnorm) {   // breakdown, or converged
          final_col_provisional = false;
          break;
        }
      }
      ncol = j + 1;
      res_next = hb[4];
      if (std::fabs(hb[4]) <= rtol * bnorm || beta == 0.0) break;
    }
    const int jn = ncol;
    givens_solve(G, GL, m, jn, final_col_provisional ? jn - 1 : -1, c->dsc + 512, s);
    combine<T>(Z, ld, jn, c->dsc + 512, x, n, s);
    if (std::is_same<T, double>::value) {
      A(reinterpret_cast<const T*>(x), yt);
    } else {
      convert<double, float>(x, reinterpret_cast<float*>(xt), n, s);
      A(xt, yt);
    }
    sub_from<T>(b, yt, c->rk, n, s);
    rn = dev_norm(c, c->rk, n, s);
    *est = rn / bnorm;
    if (rn <= rtol * bnorm) break;
    if (!std::isfinite(rn)) throw Fail{ST_IGA_ENOCONV, "non-finite residual"};
    stall.cycle(rn);
  }
  return it;
}

template <class T>
int fgmres(st_iga_ctx* c, const OpT<T>& A, const OpT<T>& Pc, const double* b, double* x, double rtol, int maxit,
           double bnorm, double* est, T* V, T* Z, T* xt, T* yt, hipStream_t s) {
  if (c->opt.reorth == 2) return fgmres_delayed<T>(c, A, Pc, b, x, rtol, maxit, bnorm, est, V, Z, xt, yt, s);
  const int64_t n = c->nunk, ld = c->ldb;
  const int m = c->opt.restart;
  const int nb = reduce_blocks(n);
  fill(x, 0.0, n, s);
  int it = 0;
  double rn = bnorm;
  Stall stall(c, bnorm, "FGMRES stagnated");
  CK(hipMemcpyAsync(c->rk, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  std::vector<double> H(static_cast<size_t>(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  double hbuf[258];
  while (it < maxit) {
    scale_to<T>(c->rk, 1.0 / rn, V, n, s);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = rn;
    int j = 0;
    for (; j < m && it < maxit; ++j) {
      T* Vj = V + static_cast<int64_t>(j) * ld;
      T* Zj = Z + static_cast<int64_t>(j) * ld;
      T* w = V + static_cast<int64_t>(j + 1) * ld;
      if (c->opt.reorth == 1 && c->opt.graphs != 0 && !kprof_enabled()) {
        // classical Gram-Schmidt twice, the whole step replayed from a HIP
        // graph (captured on first use of column j with the current ranks)
        auto body = [&](hipStream_t ss) {
          c->op_stream = ss;
          Pc(Vj, Zj);
          A(Zj, w);
          c->op_stream = s;
          multidot_partial<T>(V, ld, j + 1, w, n, c->part, nb, ss);
          finalize_sum(c->part, nb, j + 1, c->dsc, ss);
          update_norm_partial<T>(V, ld, j + 1, c->dsc, w, n, c->part, nb, ss);
          multidot_partial<T>(V, ld, j + 1, w, n, c->part, nb, ss);
          finalize_sum(c->part, nb, j + 1, c->dsc + 128, ss);
          update_norm_partial<T>(V, ld, j + 1, c->dsc + 128, w, n, c->part, nb, ss);
          finalize_sum(c->part, nb, 1, c->dsc + 256, ss);
        };
        run_step(c, c->graphs[std::is_same<T, double>::value ? 0 : 1], j, m, body, s);
        CK(hipMemcpyAsync(hbuf, c->dsc, 257 * sizeof(double), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        check_launch();
        for (int i = 0; i <= j; ++i) hbuf[66 + i] = hbuf[128 + i];
        hbuf[132] = hbuf[256];
      } else {
        Pc(Vj, Zj);
        A(Zj, w);
        // classical Gram-Schmidt; w is column j+1 of V, so the same multi-dot
        // also gives ||w||^2 before the projection
        multidot_partial<T>(V, ld, j + 2, w, n, c->part, nb, s);
        finalize_sum(c->part, nb, j + 2, c->dsc, s);
        update_norm_partial<T>(V, ld, j + 1, c->dsc, w, n, c->part, nb, s);
        finalize_sum(c->part, nb, 1, c->dsc + 256, s);
        CK(hipMemcpyAsync(hbuf, c->dsc, (j + 2) * sizeof(double), hipMemcpyDeviceToHost, s));
        CK(hipMemcpyAsync(hbuf + 132, c->dsc + 256, sizeof(double), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        check_launch();
        for (int i = 0; i <= j; ++i) hbuf[66 + i] = 0.0;
        // second pass when the first removed most of w (norm ratio below
        // 1/sqrt(2)), or always when requested
        if (c->opt.reorth != 0 || 2.0 * hbuf[132] < hbuf[j + 1]) {
          multidot_partial<T>(V, ld, j + 1, w, n, c->part, nb, s);
          finalize_sum(c->part, nb, j + 1, c->dsc + 128, s);
          update_norm_partial<T>(V, ld, j + 1, c->dsc + 128, w, n, c->part, nb, s);
          finalize_sum(c->part, nb, 1, c->dsc + 256, s);
          CK(hipMemcpyAsync(hbuf + 66, c->dsc + 128, (j + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
          CK(hipMemcpyAsync(hbuf + 132, c->dsc + 256, sizeof(double), hipMemcpyDeviceToHost, s));
          CK(hipStreamSynchronize(s));
          check_launch();
        }
      }
      ++it;
      for (int i = 0; i <= j; ++i) H[static_cast<size_t>(i) * m + j] = hbuf[i] + hbuf[66 + i];
      const double hn = std::sqrt(std::max(hbuf[132], 0.0));
      if (!std::isfinite(hn)) throw Fail{ST_IGA_ENOCONV, "non-finite Arnoldi norm"};
      scale_by_dev<T>(w, n, c->dsc + 256, s);
      for (int i = 0; i < j; ++i) {
        const double t1 = H[static_cast<size_t>(i) * m + j], t2 = H[static_cast<size_t>(i + 1) * m + j];
        H[static_cast<size_t>(i) * m + j] = cs[i] * t1 + sn[i] * t2;
        H[static_cast<size_t>(i + 1) * m + j] = -sn[i] * t1 + cs[i] * t2;
      }
      const double hjj = H[static_cast<size_t>(j) * m + j];
      const double den = std::hypot(hjj, hn);
      cs[j] = den == 0.0 ? 1.0 : hjj / den;
      sn[j] = den == 0.0 ? 0.0 : hn / den;
      H[static_cast<size_t>(j) * m + j] = den;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      if (std::fabs(g[j + 1]) <= rtol * bnorm || hn == 0.0) {
        ++j;
        break;
      }
    }
    for (int i = j - 1; i >= 0; --i) {
      double t = g[i];
      for (int k = i + 1; k < j; ++k) t -= H[static_cast<size_t>(i) * m + k] * y[k];
      y[i] = t / H[static_cast<size_t>(i) * m + i];
    }
    CK(hipMemcpyAsync(c->dsc + 512, y.data(), j * sizeof(double), hipMemcpyHostToDevice, s));
    combine<T>(Z, ld, j, c->dsc + 512, x, n, s);
    // restart residual r = b - A x with the same operator
    if (std::is_same<T, double>::value) {
      A(reinterpret_cast<const T*>(x), yt);
    } else {
      convert<double, float>(x, reinterpret_cast<float*>(xt), n, s);
      A(xt, yt);
    }
    sub_from<T>(b, yt, c->rk, n, s);
    rn = dev_norm(c, c->rk, n, s);
    *est = rn / bnorm;
    if (rn <= rtol * bnorm) break;
    if (!std::isfinite(rn)) throw Fail{ST_IGA_ENOCONV, "non-finite residual"};
    stall.cycle(rn);
  }
  return it;
}

void ensure_lin(st_iga_ctx* c) {
  if (!c->linearized) throw Fail{ST_IGA_ESTATE, "no linearization set (call st_iga_linearize or st_iga_set_factors)"};
}

void apply64(st_iga_ctx* c, const double* x, double* y, hipStream_t s) {
  Bufs<double> B = bufs64(c);
  apply_impl<double, double>(c, x, y, c->Nt, 1, true, true, B, s);
}
void precond64(st_iga_ctx* c, const double* r, double* z, hipStream_t s) {
  Bufs<double> B = bufs64(c);
  precond_impl<double, double>(c, r, z, B, s);
}

template <class S>
void lowp_ops(st_iga_ctx* c, Op& A, Op& Pc, hipStream_t s);

template <>
void lowp_ops<float>(st_iga_ctx* c, Op& A, Op& Pc, hipStream_t s) {
  A = [c, s](const double* x, double* y) {
    Bufs<float> B;
    for (int k = 0; k < 4; ++k) B.t4[k] = c->t4f[k];
    B.big[0] = c->bigf[0];
    B.big[1] = c->bigf[1];
    B.Psi = c->Psi_f;
    convert<double, float>(x, c->xf, c->nunk, s);
    apply_impl<float, float>(c, c->xf, c->yf, c->Nt, 1, true, true, B, s);
    convert<float, double>(c->yf, y, c->nunk, s);
  };
  Pc = [c, s](const double* r, double* z) {
    Bufs<float> B;
    for (int k = 0; k < 4; ++k) B.t4[k] = c->t4f[k];
    B.big[0] = c->bigf[0];
    B.big[1] = c->bigf[1];
    B.Psi = c->Psi_f;
    convert<double, float>(r, c->xf, c->nunk, s);
    precond_impl<float, float>(c, c->xf, c->yf, B, s);
    convert<float, double>(c->yf, z, c->nunk, s);
  };
}
// BF16 mode: the operator stays FP32 (BF16 rounding of the operator makes
// iterative refinement non-contractive on these systems); the preconditioner's
// mode products and arrowhead run with BF16 storage and FP32 arithmetic.
template <>
void lowp_ops<bf16>(st_iga_ctx* c, Op& A, Op& Pc, hipStream_t s) {
  Op unused;
  lowp_ops<float>(c, A, unused, s);
  Pc = [c, s](const double* r, double* z) {
    Bufs<bf16> B;
    for (int k = 0; k < 4; ++k) B.t4[k] = c->t4b[k];
    B.big[0] = B.big[1] = nullptr;
    B.Psi = nullptr;
    convert<double, bf16>(r, c->xb, c->nunk, s);
    precond_impl<bf16, float>(c, c->xb, c->yb, B, s);
    convert<bf16, double>(c->yb, z, c->nunk, s);
  };
}

// Low-precision operators on FP32 buffers for the inner solves.
void lowp_ops_f32(st_iga_ctx* c, OpT<float>& A, OpT<float>& Pc, hipStream_t s) {
  c->op_stream = s;
  A = [c](const float* x, float* y) {
    const hipStream_t s = c->op_stream;
    Bufs<float> B;
    for (int k = 0; k < 4; ++k) B.t4[k] = c->t4f[k];
    B.big[0] = c->bigf[0];
    B.big[1] = c->bigf[1];
    B.Psi = c->Psi_f;
    apply_impl<float, float>(c, x, y, c->Nt, 1, true, true, B, s);
  };
  if (c->opt.prec == ST_IGA_MIXED_FP32) {
    Pc = [c](const float* r, float* z) {
      const hipStream_t s = c->op_stream;
      Bufs<float> B;
      for (int k = 0; k < 4; ++k) B.t4[k] = c->t4f[k];
      B.big[0] = c->bigf[0];
      B.big[1] = c->bigf[1];
      B.Psi = c->Psi_f;
      precond_impl<float, float>(c, r, z, B, s);
    };
  } else {
    Pc = [c](const float* r, float* z) {
      const hipStream_t s = c->op_stream;
      Bufs<bf16> B;
      for (int k = 0; k < 4; ++k) B.t4[k] = c->t4b[k];
      B.big[0] = B.big[1] = nullptr;
      B.Psi = nullptr;
      convert<float, bf16>(r, c->xb, c->nunk, s);
      precond_impl<bf16, float>(c, c->xb, c->yb, B, s);
      convert<bf16, float>(c->yb, z, c->nunk, s);
    };
  }
}

// Linear solve with the configured precision.  Returns iterations.
int krylov(st_iga_ctx* c, const double* b, double* x, double tol, double* relres, hipStream_t s) {
  ensure_lin(c);
  const int64_t n = c->nunk;
  const double bnorm = dev_norm(c, b, n, s);
  if (bnorm == 0.0) {
    fill(x, 0.0, n, s);
    *relres = 0.0;
    return 0;
  }
  double est = 1.0;
  if (c->opt.prec == ST_IGA_FP64) {
    c->op_stream = s;
    OpT<double> A64 = [c](const double* xx, double* yy) { apply64(c, xx, yy, c->op_stream); };
    OpT<double> P64 = [c](const double* rr, double* zz) { precond64(c, rr, zz, c->op_stream); };
    const int it = fgmres<double>(c, A64, P64, b, x, tol, c->opt.max_krylov, bnorm, &est,
                                  static_cast<double*>(c->Vb), static_cast<double*>(c->Zb), nullptr, c->wk, s);
    *relres = est;
    if (est > tol) throw Fail{ST_IGA_ENOCONV, "FGMRES reached max_krylov"};
    return it;
  }
  OpT<float> Al, Pl;
  lowp_ops_f32(c, Al, Pl, s);
  // iterative refinement on the FP64 true residual
  fill(x, 0.0, n, s);
  CK(hipMemcpyAsync(c->bk, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));   // bk = current residual
  double rn = bnorm;
  int total = 0, refinements = 0;
  Stall stall(c, bnorm, "iterative refinement stagnated");
  while (rn > tol * bnorm) {
    if (total >= c->opt.max_krylov || refinements >= 60) throw Fail{ST_IGA_ENOCONV, "refinement did not converge"};
    const double itol = std::max(c->opt.inner_tol, 0.5 * tol * bnorm / rn);
    double e2 = 1.0;
    total += fgmres<float>(c, Al, Pl, c->bk, c->dk, itol, c->opt.max_krylov - total, rn, &e2,
                           static_cast<float*>(c->Vb), static_cast<float*>(c->Zb), c->xf, c->yf, s);
    axpy(1.0, c->dk, x, n, s);
    apply64(c, x, c->wk, s);
    axpby(1.0, b, -1.0, c->wk, n, s);
    CK(hipMemcpyAsync(c->bk, c->wk, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    rn = dev_norm(c, c->bk, n, s);
    ++refinements;
    if (!std::isfinite(rn)) throw Fail{ST_IGA_ENOCONV, "non-finite residual"};
    if (rn > tol * bnorm) stall.cycle(rn);
  }
  c->last_refinements = refinements;
  *relres = rn / bnorm;
  return total;
}

// ------------------------------------------------------------------ linearization
// Spatial expansion of an array [L][n_d..n_1] with per-axis tables into dst [L][Q_d..Q_1].
void expand_space(st_iga_ctx* c, const Tab* const* tabs, const double* x, int64_t L, double* tA, double* tB, double* dst,
                  double alpha, double beta, hipStream_t s) {
  const int nn[3] = {c->n[0], c->n[1], c->n[2]};
  const int qd[3] = {c->Q[0], c->Q[1], c->Q[2]};
  if (c->d == 1) {
    gather<double, double, double>(tabs[0]->d, x, dst, L, 1, nn[0], 0, alpha, beta, s);
    return;
  }
  spatial_chain<double, double>(c, tabs, x, L, nn, qd, tA, tB, dst, alpha, beta, s);
}
void project_space(st_iga_ctx* c, const double* g, int64_t L, double* tA, double* tB, double* dst, double beta,
                   hipStream_t s) {
  const int nn[3] = {c->n[0], c->n[1], c->n[2]};
  const int qd[3] = {c->Q[0], c->Q[1], c->Q[2]};
  const Tab* pr[3] = {&c->BqT[0], &c->BqT[1], &c->BqT[2]};
  if (c->d == 1) {
    gather<double, double, double>(pr[0]->d, g, dst, L, 1, qd[0], 0, 1.0, beta, s);
    return;
  }
  spatial_chain<double, double>(c, pr, g, L, qd, nn, tA, tB, dst, 1.0, beta, s);
}

// Maxima of |u| and |u_t| from nb interleaved block partials in part; the
// two maxima go to dsc[300], dsc[301].
void finish_uv_maxima(st_iga_ctx* c, int64_t nb, hipStream_t s) {
  finalize_max2(c->part, nb, c->dsc + 300, s);
  check_launch();
}

// The quadrature pass with the slowest spatial axis fused (d >= 2): per
// chunk of time elements, time gathers, expansions along the faster axes,
// one k_quad_fused launch, then the element-maxima reductions and the
// projection of the ionic current back to the B-splines.
void quad_pass_fused(st_iga_ctx* c, const double* u, const double* w, bool want_res, bool want_theta,
                     hipStream_t s) {
  const int d = c->d;
  const st_iga_problem& P = c->P;
  const int64_t Ns = c->Ns;
  const int nq = c->nqt;
  const int nd = c->n[d - 1], neld = c->nel[d - 1];
  const int64_t Qin = (d == 3) ? static_cast<int64_t>(c->Q[0]) * c->Q[1] : c->Q[0];
  const int64_t L2 = static_cast<int64_t>(nd) * Qin;
  const int64_t X1 = (d == 3) ? static_cast<int64_t>(c->n[2]) * c->n[1] * c->Q[0] : 0;
  const int ne_max = c->qf_ne;
  const int64_t rmax = static_cast<int64_t>(ne_max) * nq;
  if (rmax * (3 * Ns + 4 * X1) > c->big_len || rmax * 6 * L2 + 2LL * ne_max * neld * Qin > c->big_len)
    throw Fail{ST_IGA_EDEVICE, "quadrature chunk does not fit"};
  double* U0 = c->big[0];
  double* Ut = U0 + rmax * Ns;
  double* W0 = Ut + rmax * Ns;
  double* Xa = W0 + rmax * Ns;              // 3D: x1 expansions a, b, u_t, w
  double* Xb = Xa + rmax * X1;
  double* Xt = Xb + rmax * X1;
  double* Xw = Xt + rmax * X1;
  double* in[5];
  for (int k = 0; k < 5; ++k) in[k] = c->big[1] + k * rmax * L2;
  double* Gp = c->big[1] + 5 * rmax * L2;
  double* Mp = Gp + rmax * L2;
  double* Mx = Mp + static_cast<int64_t>(ne_max) * neld * Qin;
  if (want_res) fill(c->rfull, 0.0, c->nfull, s);
  const int n1 = c->n[0], n2 = c->n[1], n3 = c->n[2], Q1 = c->Q[0], Q2 = c->Q[1];
  auto ax = [&](const Tab& t, const double* xin, double* yout, int64_t outer, int64_t inner, int nin) {
    gather<double, double, double>(t.d, xin, yout, outer, inner, nin, 0, 1.0, 0.0, s);
  };
  int64_t boff = 0;
  for (int e0 = 0; e0 < c->nelt; e0 += ne_max) {
    const int ne = std::min(ne_max, c->nelt - e0);
    const int q0 = e0 * nq, nqc = ne * nq;
    gather_rows<double, double, double>(c->Bt0.d, q0, nqc, u, U0, 1, Ns, c->nt, 0, 1.0, 0.0, s);
    gather_rows<double, double, double>(c->Bt1.d, q0, nqc, u, Ut, 1, Ns, c->nt, 0, 1.0, 0.0, s);
    gather_rows<double, double, double>(c->Bt0.d, q0, nqc, w, W0, 1, Ns, c->nt, 0, 1.0, 0.0, s);
    const Tab &E0 = c->Bq[0][0], &E2 = c->Bq[0][2];
    double sL, sM, sF;
    if (d == 3) {
      const Tab &F0 = c->Bq[1][0], &F2 = c->Bq[1][2];
      const int64_t o1 = static_cast<int64_t>(nqc) * n3 * n2, o2 = static_cast<int64_t>(nqc) * n3;
      ax(E0, U0, Xa, o1, 1, n1);
      ax(E2, U0, Xb, o1, 1, n1);
      ax(E0, Ut, Xt, o1, 1, n1);
      ax(E0, W0, Xw, o1, 1, n1);
      if (!c->qf_x2) {
        ax(F0, Xa, in[0], o2, Q1, n2);   // B0 B0 u
        ax(F2, Xa, in[1], o2, Q1, n2);   // x2 second derivative
        ax(F0, Xb, in[2], o2, Q1, n2);   // x1 second derivative
        ax(F0, Xt, in[3], o2, Q1, n2);
        ax(F0, Xw, in[4], o2, Q1, n2);
      }
      sL = P.sigma[2];
      sM = P.sigma[1];
      sF = P.sigma[0];
    } else {
      const int64_t o1 = static_cast<int64_t>(nqc) * n2;
      ax(E0, U0, in[0], o1, 1, n1);
      ax(E2, U0, in[2], o1, 1, n1);
      ax(E0, Ut, in[3], o1, 1, n1);
      ax(E0, W0, in[4], o1, 1, n1);
      sL = P.sigma[1];
      sM = 0.0;
      sF = P.sigma[0];
    }
    const bool x2 = d == 3 && c->qf_x2;
    const DTable<double> &F0d = c->Bq[1][0].d, &F2d = c->Bq[1][2].d;
    const int64_t nb =
        x2 ? quad_fused(d, P.p_s, nq, Xa, nullptr, Xb, Xt, Xw, nd, Qin, ne, c->cf_Bl_d, c->cf_B2_d, c->cf_first,
                        c->cf_chunks, c->cf_nchunk, c->wq_t + q0, c->qf_win, c->qf_wd, sL, sM, sF, P.Cm, P.a, P.c1,
                        P.c2, want_res ? Gp : nullptr, want_theta ? Mp : nullptr, neld, c->part, boff, s, n2, Q1,
                        F0d.coef, F2d.coef, F0d.c0, c->src, q0, c->cq_out, c->rq_out, c->Qs)
           : quad_fused(d, P.p_s, nq, in[0], in[1], in[2], in[3], in[4], nd, Qin, ne, c->cf_Bl_d, c->cf_B2_d,
                        c->cf_first, c->cf_chunks, c->cf_nchunk, c->wq_t + q0, c->qf_win, c->qf_wd, sL, sM, sF, P.Cm,
                        P.a, P.c1, P.c2, want_res ? Gp : nullptr, want_theta ? Mp : nullptr, neld, c->part, boff, s,
                        0, 1, nullptr, nullptr, nullptr, c->src, q0, c->cq_out, c->rq_out, c->Qs);
    if (nb < 0) throw Fail{ST_IGA_EINVAL, "fused quadrature pass: unsupported degrees"};
    boff += nb;
    if (want_theta) {
      double* Edst = c->E + static_cast<int64_t>(e0) * c->Nels;
      if (d == 3) {
        mode_max(c->el_s_s[0], c->el_s_c[0], c->nel[0], Mp, Mx, static_cast<int64_t>(ne) * neld * Q2, 1, Q1, s);
        mode_max(c->el_s_s[1], c->el_s_c[1], c->nel[1], Mx, Edst, static_cast<int64_t>(ne) * neld, c->nel[0], Q2, s);
      } else {
        mode_max(c->el_s_s[0], c->el_s_c[0], c->nel[0], Mp, Edst, static_cast<int64_t>(ne) * neld, 1, Q1, s);
      }
    }
    if (want_res) {
      if (d == 3) {
        ax(c->BqT[1], Gp, Xa, static_cast<int64_t>(nqc) * n3, Q1, Q2);
        ax(c->BqT[0], Xa, U0, static_cast<int64_t>(nqc) * n3 * n2, 1, Q1);
      } else {
        ax(c->BqT[0], Gp, U0, static_cast<int64_t>(nqc) * n2, 1, Q1);
      }
      gather<double, double, double>((c->supg ? c->BtTs : c->BtT).d, U0, c->rfull, 1, Ns, nqc, q0, 1.0, 1.0, s);
    }
  }
  finish_uv_maxima(c, boff, s);
}

// One pass over all space-time Gauss points (time-chunked): ionic part of the
// residual into rfull (full rows) and/or the element maxima of |R| into E; the
// maxima of |u| and |u_t| into dsc[300], dsc[301].
void quad_pass(st_iga_ctx* c, const double* u, const double* w, bool want_res, bool want_theta, hipStream_t s) {
  if (c->qf) {
    quad_pass_fused(c, u, w, want_res, want_theta, s);
    return;
  }
  const int d = c->d;
  const st_iga_problem& P = c->P;
  const int64_t Ns = c->Ns, Qs = c->Qs;
  const int nq = c->nqt;
  double* pool = c->big[0];    // both big buffers are contiguous-enough scratch: carve sequentially
  const int64_t cq = static_cast<int64_t>(c->chunk_el) * nq;
  double* U0 = pool;
  double* Ut = U0 + cq * Ns;
  double* W0 = Ut + cq * Ns;
  double* uq = c->big[1];
  double* utq = uq + cq * Qs;
  double* wq = utq + cq * Qs;
  double* lap = wq + cq * Qs;
  double* g = W0 + cq * Ns;          // in big[0] after W0
  double* absR = g + cq * Qs;
  double* tA = absR + cq * Qs;
  double* tB = lap + cq * Qs;        // in big[1]
  // capacity check (both regions hold nt*Qs doubles)
  const int64_t capb = c->big_len;
  if (3 * cq * Ns + 3 * cq * Qs > capb || 5 * cq * Qs > capb) throw Fail{ST_IGA_EDEVICE, "quadrature chunk does not fit"};
  if (want_res) fill(c->rfull, 0.0, c->nfull, s);
  const Tab* B0[3] = {&c->Bq[0][0], &c->Bq[1][0], &c->Bq[2][0]};
  int boff = 0;
  double* part_u = c->part;
  double* part_t = c->part + c->nb_part;
  const int nel_s[3] = {c->nel[0], c->nel[1], c->nel[2]};
  for (int e0 = 0; e0 < c->nelt; e0 += c->chunk_el) {
    const int ne = std::min(c->chunk_el, c->nelt - e0);
    const int q0 = e0 * nq, nqc = ne * nq;
    gather_rows<double, double, double>(c->Bt0.d, q0, nqc, u, U0, 1, Ns, c->nt, 0, 1.0, 0.0, s);
    gather_rows<double, double, double>(c->Bt1.d, q0, nqc, u, Ut, 1, Ns, c->nt, 0, 1.0, 0.0, s);
    gather_rows<double, double, double>(c->Bt0.d, q0, nqc, w, W0, 1, Ns, c->nt, 0, 1.0, 0.0, s);
    expand_space(c, B0, Ut, nqc, tA, tB, utq, 1.0, 0.0, s);
    expand_space(c, B0, W0, nqc, tA, tB, wq, 1.0, 0.0, s);
    // u and sum_l sigma_l d_ll u with shared partial expansions (g and absR
    // are free until the pointwise kernel)
    {
      const int n1 = c->n[0], n2 = c->n[1], n3 = c->n[2], Q1 = c->Q[0], Q2 = c->Q[1];
      auto ax = [&](const Tab& t, const double* xin, double* yout, int64_t outer, int64_t inner, int nin, double al,
                    double be) { gather<double, double, double>(t.d, xin, yout, outer, inner, nin, 0, al, be, s); };
      const Tab &E0 = c->Bq[0][0], &E2 = c->Bq[0][2];
      if (d == 1) {
        ax(E0, U0, uq, nqc, 1, n1, 1.0, 0.0);
        ax(E2, U0, lap, nqc, 1, n1, P.sigma[0], 0.0);
      } else if (d == 2) {
        const Tab &F0 = c->Bq[1][0], &F2 = c->Bq[1][2];
        ax(E0, U0, tA, static_cast<int64_t>(nqc) * n2, 1, n1, 1.0, 0.0);       // a = B0 x1
        ax(E2, U0, tB, static_cast<int64_t>(nqc) * n2, 1, n1, 1.0, 0.0);       // b = B2 x1
        ax(F0, tA, uq, nqc, Q1, n2, 1.0, 0.0);
        ax(F2, tA, lap, nqc, Q1, n2, P.sigma[1], 0.0);
        ax(F0, tB, lap, nqc, Q1, n2, P.sigma[0], 1.0);
      } else {
        const Tab &F0 = c->Bq[1][0], &F2 = c->Bq[1][2], &G0 = c->Bq[2][0], &G2 = c->Bq[2][2];
        const int64_t o1 = static_cast<int64_t>(nqc) * n3 * n2, o2 = static_cast<int64_t>(nqc) * n3;
        ax(E0, U0, tA, o1, 1, n1, 1.0, 0.0);                    // a  = B0 x1
        ax(E2, U0, tB, o1, 1, n1, 1.0, 0.0);                    // b  = B2 x1
        ax(F0, tA, g, o2, Q1, n2, 1.0, 0.0);                    // aa = B0 x2 a
        ax(F2, tA, absR, o2, Q1, n2, 1.0, 0.0);                 // ab = B2 x2 a
        ax(F0, tB, tA, o2, Q1, n2, 1.0, 0.0);                   // ba = B0 x2 b
        const int64_t in3 = static_cast<int64_t>(Q1) * Q2;
        ax(G0, g, uq, nqc, in3, n3, 1.0, 0.0);
        ax(G2, g, lap, nqc, in3, n3, P.sigma[2], 0.0);
        ax(G0, absR, lap, nqc, in3, n3, P.sigma[1], 1.0);
        ax(G0, tA, lap, nqc, in3, n3, P.sigma[0], 1.0);
      }
    }
    const int nbp = static_cast<int>((static_cast<int64_t>(nqc) * Qs + 255) / 256);
    pointwise_ionic(uq, utq, lap, wq, c->wq_t + q0, c->wq_s, Qs, nqc, P.Cm, P.a, P.c1, P.c2, g, absR,
                    part_u + boff, nbp, s, c->src, q0, c->Q[0], c->Q[1], c->cq_out, c->rq_out);
    // the kernel writes [2b], [2b+1] pairs: keep them interleaved in part_u region
    boff += 2 * nbp;
    if (want_theta) {
      // element maxima: time axis (within chunk), then spatial axes
      double* cur = absR;
      int dims[4];
      dims[0] = nqc;
      for (int l = 0; l < d; ++l) dims[1 + l] = c->Q[l];
      // time axis: [nqc][Qs] -> [ne][Qs]
      mode_max(c->el_t_s, c->el_t_c, ne, cur, tA, 1, Qs, nqc, s);
      cur = tA;
      dims[0] = ne;
      double* nxt = tB;
      for (int l = 0; l < d; ++l) {
        int64_t inner = 1, outer = ne;
        for (int k = 0; k < l; ++k) inner *= nel_s[k];
        for (int k = l + 1; k < d; ++k) outer *= c->Q[k];
        double* out = (l == d - 1) ? c->E + static_cast<int64_t>(e0) * c->Nels : nxt;
        mode_max(c->el_s_s[l], c->el_s_c[l], nel_s[l], cur, out, outer, inner, c->Q[l], s);
        nxt = cur;
        cur = out;
      }
    }
    if (want_res) {
      // project g over space into U0 region (reuse), then over time into rfull
      project_space(c, g, nqc, tA, tB, U0, 0.0, s);
      DTable<double> tt = (c->supg ? c->BtTs : c->BtT).d;   // test functions b_i (+ tau b_i' with SUPG)
      gather<double, double, double>(tt, U0, c->rfull, 1, Ns, nqc, q0, 1.0, 1.0, s);
    }
  }
  (void)part_t;
  // maxima of |u| and |u_t| from the interleaved partials ([2b] |u|, [2b+1] |u_t|)
  finish_uv_maxima(c, boff / 2, s);
}

// Theta grid (N_t x N_s) of eq. (3.6) into dst.
void theta_grid(st_iga_ctx* c, const double* u, const double* w, double* dst, hipStream_t s, bool with_res = false) {
  const int d = c->d;
  quad_pass(c, u, w, with_res, true, s);
  // window maxima: time then spatial axes; E is [nelt][nel_d..nel_1]
  double* tA = c->big[0];
  double* tB = c->big[1];
  mode_max(c->win_t_s, c->win_t_c, c->Nt, c->E, tA, 1, c->Nels, c->nelt, s);
  int dims[3] = {c->nel[0], c->nel[1], c->nel[2]};
  double* cur = tA;
  for (int l = 0; l < d; ++l) {
    int64_t inner = 1, outer = c->Nt;
    for (int k = 0; k < l; ++k) inner *= c->n[k];
    for (int k = l + 1; k < d; ++k) outer *= dims[k];
    double* out = (l == d - 1) ? dst : (cur == tA ? tB : tA);
    mode_max(c->win_s_s[l], c->win_s_c[l], c->n[l], cur, out, outer, inner, dims[l], s);
    dims[l] = c->n[l];
    cur = out;
  }
  theta_finish(dst, c->nunk, c->dsc + 300, c->P.Cm, 1.0 / c->P.T, s);
  check_launch();
}

// Values at the (X_t time) x (space) Greville grid of a full vector.
void greville_values(st_iga_ctx* c, const double* x, double* dst, hipStream_t s) {
  const int d = c->d;
  const int64_t Ns = c->Ns;
  double* tA = c->t4[2];
  double* tB = c->t4[3];
  // time first: [n_t][Ns] -> [N_t][Ns]
  gather<double, double, double>(c->Gt.d, x, tA, 1, Ns, c->nt, 0, 1.0, 0.0, s);
  const Tab* G[3] = {&c->Gs[0], &c->Gs[1], &c->Gs[2]};
  const int nn[3] = {c->n[0], c->n[1], c->n[2]};
  if (d == 1) {
    gather<double, double, double>(G[0]->d, tA, dst, c->Nt, 1, nn[0], 0, 1.0, 0.0, s);
    return;
  }
  spatial_chain<double, double>(c, G, tA, c->Nt, nn, nn, tB, tA, dst, 1.0, 0.0, s);
}

// Truncated SVD of an N_t x N_s device matrix through its Gram matrix.
// Returns R; U (N_t x R, host), s (host), V (device N_s x R, into Vdst).
int lowrank(st_iga_ctx* c, const double* C, double eps, std::vector<double>& U, std::vector<double>& sv, double* Vdst,
            hipStream_t s) {
  const int m = c->Nt;
  const int64_t n = c->Ns;
  gram_partial(C, m, n, c->gram, c->gram_nb, s);
  finalize_sum(c->gram, c->gram_nb, m * m, c->big[0], s);
  std::vector<double> G(static_cast<size_t>(m) * m);
  CK(hipMemcpyAsync(G.data(), c->big[0], G.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  check_launch();
  std::vector<double> Q, lam;
  std::string err;
  if (!sym_eig(G, m, Q, lam, err)) {
    // the QL iteration failing on finite data is not expected; Jacobi sweeps
    // (slower, unconditionally convergent) are the fallback
    if (err == "non-finite matrix entry") throw Fail{ST_IGA_ENOCONV, "Gram matrix of the low rank is not finite"};
    std::vector<double> I(static_cast<size_t>(m) * m, 0.0);
    for (int i = 0; i < m; ++i) I[static_cast<size_t>(i) * m + i] = 1.0;
    if (!gen_eig_sym(G, I, m, Q, lam, err)) throw Fail{ST_IGA_EDEVICE, "Gram eigendecomposition: " + err};
  }
  // descending order
  double tot = 0.0;
  for (double& v : lam) { v = std::max(v, 0.0); tot += v; }
  c->lr_relerr = 0.0;
  c->lr_capped = false;
  if (tot == 0.0) { U.clear(); sv.clear(); return 0; }
  std::vector<int> idx(m);
  for (int i = 0; i < m; ++i) idx[i] = m - 1 - i;
  int R = m;
  double tail = 0.0;
  // smallest R with sum_{k >= R} lam_k <= eps^2 tot
  for (int r = m; r >= 0; --r) {
    if (r < m) tail += lam[idx[r]];
    if (tail <= eps * eps * tot) R = r;
    else break;
  }
  const int Rtol = R;
  if (R > c->maxR) R = c->maxR;   // capped: the tolerance is then not met (flagged in the report)
  {
    double t = 0.0;
    for (int r = R; r < m; ++r) t += lam[idx[r]];
    c->lr_relerr = std::sqrt(t / tot);
    c->lr_capped = Rtol > R;
  }
  U.assign(static_cast<size_t>(m) * R, 0.0);
  sv.assign(R, 0.0);
  std::vector<double> inv(R);
  for (int r = 0; r < R; ++r) {
    sv[r] = std::sqrt(lam[idx[r]]);
    inv[r] = 1.0 / sv[r];
    for (int i = 0; i < m; ++i) U[static_cast<size_t>(i) * R + r] = Q[static_cast<size_t>(i) * m + idx[r]];
  }
  if (R > 0) {
    CK(hipMemcpyAsync(c->tmpR, U.data(), U.size() * sizeof(double), hipMemcpyHostToDevice, s));
    CK(hipMemcpyAsync(c->tmpR + static_cast<int64_t>(m) * c->maxR, inv.data(), R * sizeof(double), hipMemcpyHostToDevice, s));
    right_factor(C, m, n, c->tmpR, c->tmpR + static_cast<int64_t>(m) * c->maxR, R, Vdst, s);
    CK(hipStreamSynchronize(s));
    check_launch();
  }
  return R;
}

// Rebuild Psi (spatial factors at Gauss points times weights) and the time
// tables T_r for both factor sets: theta in [0, Rth), reaction in [Rth, Rth+Rc).
void rebuild_coefficients(st_iga_ctx* c, hipStream_t s) {
  const int d = c->d;
  const st_iga_problem& P = c->P;
  const Dir1D& T = c->dir[d];
  const int Nt = c->Nt, pt = P.p_t, WB = 2 * pt + 1;
  const int Rt = c->Rth + c->Rc;
  // spatial factors
  const Tab* Hs[3] = {&c->Hs[0], &c->Hs[1], &c->Hs[2]};
  const int nn[3] = {c->n[0], c->n[1], c->n[2]};
  const int qd[3] = {c->Q[0], c->Q[1], c->Q[2]};
  for (int set = 0; set < 2; ++set) {
    const int R = set == 0 ? c->Rth : c->Rc;
    if (R == 0) continue;
    const double* V = set == 0 ? c->Vth : c->Vc;
    double* dst = c->Psi + static_cast<int64_t>(set == 0 ? 0 : c->Rth) * c->Qs;
    transpose_nr(V, c->Ns, R, c->VT, s);
    for (int r = 0; r < R; ++r) {
      const double* src = c->VT + static_cast<int64_t>(r) * c->Ns;
      double* out = dst + static_cast<int64_t>(r) * c->Qs;
      if (d == 1) gather<double, double, double>(Hs[0]->d, src, out, 1, 1, nn[0], 0, 1.0, 0.0, s);
      else spatial_chain<double, double>(c, Hs, src, 1, nn, qd, c->big[1], c->big[1] + c->Qs, out, 1.0, 0.0, s);
    }
  }
  scale_rows(c->Psi, Rt, c->Qs, c->wq_s, s);
  if (c->Psi_f) convert<double, float>(c->Psi, c->Psi_f, static_cast<int64_t>(Rt) * c->Qs, s);
  // banded preconditioner: spatial means of the low-rank spatial factors
  // (Psi carries the Gauss weights), for the time profiles of theta and of
  // the reaction coefficient
  std::vector<double> psibar(static_cast<size_t>(std::max(Rt, 1)), 0.0);
  if (c->banded && Rt > 0) {
    row_sums(c->Psi, Rt, c->Qs, c->rowsum_d, s);
    CK(hipMemcpyAsync(psibar.data(), c->rowsum_d, Rt * sizeof(double), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    const double vol = space_volume(c);
    for (double& v : psibar) v /= vol;
  }
  if (c->banded) {
    if (c->opt.su == 1) c->prof_th.assign(T.Q, 0.0);
    if (!c->exact_react) c->prof_cr.assign(T.Q, 0.0);
  }
  // time tables
  std::vector<double> nodes(T.grev.begin() + 1, T.grev.end());
  std::vector<int> left;
  std::vector<double> wl;
  hat_weights(nodes, T.xq, left, wl);
  const int NtP = c->NtP;
  std::vector<double> Tr(static_cast<size_t>(std::max(Rt, 1)) * NtP * WB, 0.0);
  for (int set = 0; set < 2; ++set) {
    const int R = set == 0 ? c->Rth : c->Rc;
    const std::vector<double>& U = set == 0 ? c->Uth_h : c->Uc_h;
    const std::vector<double>& sv = set == 0 ? c->sth_h : c->sc_h;
    const int roff = set == 0 ? 0 : c->Rth;
    std::vector<double>* prof = !c->banded ? nullptr : set == 0 ? &c->prof_th : (c->exact_react ? nullptr : &c->prof_cr);
    for (int r = 0; r < R; ++r) {
      double* Trr = &Tr[static_cast<size_t>(roff + r) * NtP * WB];
      for (int q = 0; q < T.Q; ++q) {
        const int g0 = left[q];
        const int g1 = std::min(g0 + 1, Nt - 1);
        const double phi = wl[q] * U[static_cast<size_t>(g0) * R + r] + (1.0 - wl[q]) * U[static_cast<size_t>(g1) * R + r];
        if (prof && !prof->empty()) (*prof)[q] += sv[r] * phi * psibar[roff + r];
        const int f = T.first[q];
        for (int a = 0; a <= pt; ++a) {
          const int i = f + a;             // full row index
          if (i < 1) continue;             // rows of X_t only
          for (int bb = 0; bb <= pt; ++bb) {
            const int j = f + bb;          // full column
            const int w = j - i + pt;      // = j - (i - pt); row t = i - 1 has window start (t+1) - pt
            double val;
            if (set == 0) {
              val = 0.0;
              for (int k = 1; k <= pt; ++k)
                val += c->tauq[static_cast<size_t>(k - 1) * T.Q + q] * T.B[k][static_cast<size_t>(q) * (pt + 1) + a] *
                       T.B[k][static_cast<size_t>(q) * (pt + 1) + bb];
              val *= P.Cm;
            } else {
              val = T.B[0][static_cast<size_t>(q) * (pt + 1) + a] * T.B[0][static_cast<size_t>(q) * (pt + 1) + bb];
            }
            Trr[static_cast<size_t>(i - 1) * WB + w] += sv[r] * T.wq[q] * phi * val;
          }
        }
      }
    }
  }
  std::vector<float> Trf(Tr.begin(), Tr.end());
  CK(hipMemcpyAsync(c->Tr, Tr.data(), Tr.size() * sizeof(double), hipMemcpyHostToDevice, s));
  CK(hipMemcpyAsync(c->Tr_f, Trf.data(), Trf.size() * sizeof(float), hipMemcpyHostToDevice, s));
  CK(hipStreamSynchronize(s));
  check_launch();
  if (c->banded) time_factor(c, s);
  c->linearized = true;
}

void linearize(st_iga_ctx* c, const double* u, const double* w, bool refresh_theta, hipStream_t s,
               bool with_residual = false) {
  const bool newton = c->opt.outer == 0;
  c->rfull_u = c->rfull_w = nullptr;
  // exact C_r: the quadrature pass at (u, w) also writes omega C_r at every Gauss point
  c->cq_out = c->exact_react ? c->Cq_d : nullptr;
  c->rq_out = c->sc_on ? c->Rq_d : nullptr;   // omega |R| for the shock-capturing coefficient
  struct ClearCq {
    st_iga_ctx* c;
    ~ClearCq() { c->cq_out = c->rq_out = nullptr; }
  } clear_cq{c};
  bool cq_done = false;
  if (c->opt.su == 1 && refresh_theta) {
    // one quadrature pass gives the theta maxima and, on request, the ionic
    // part of the residual at the same (u, w)
    theta_grid(c, u, w, c->grid, s, with_residual);
    if (with_residual) {
      c->rfull_u = u;
      c->rfull_w = w;
    }
    cq_done = true;
    c->Rth = lowrank(c, c->grid, c->opt.eps_theta, c->Uth_h, c->sth_h, c->Vth, s);
    c->err_th = c->lr_relerr;
    c->cap_th = c->lr_capped;
  } else if (c->opt.su != 1) {
    c->Rth = 0;
    c->err_th = 0.0;
    c->cap_th = false;
  }
  if (c->exact_react) {
    if (!cq_done) {
      quad_pass(c, u, w, with_residual, false, s);
      if (with_residual) {
        c->rfull_u = u;
        c->rfull_w = w;
      }
    }
    const int64_t nq = static_cast<int64_t>(c->dir[c->d].Q) * c->Qs;
    if (c->Cq_f) convert<double, float>(c->Cq_d, c->Cq_f, nq, s);
    if (c->sc_on) {
      // sc_c h^2/4 |R| / (C_m (||u||/T + ||u_t||)) with the maxima of this pass
      sc_scale(c->Rq_d, c->scfac_d, c->dsc + 300, c->P.Cm, 1.0 / c->P.T, c->Qs, nq, s);
      if (c->Rq_f) convert<double, float>(c->Rq_d, c->Rq_f, nq, s);
    }
    if (c->banded) {
      // spatial means of C_r and of the shock-capturing coefficient at each
      // time Gauss point (Cq and Rq carry the Gauss weights)
      const Dir1D& T = c->dir[c->d];
      row_sums(c->Cq_d, T.Q, c->Qs, c->rowsum_d, s);
      if (c->sc_on) row_sums(c->Rq_d, T.Q, c->Qs, c->rowsum_d + T.Q, s);
      std::vector<double> sums(2 * static_cast<size_t>(T.Q), 0.0);
      CK(hipMemcpyAsync(sums.data(), c->rowsum_d, (c->sc_on ? 2 : 1) * T.Q * sizeof(double), hipMemcpyDeviceToHost,
                        s));
      CK(hipStreamSynchronize(s));
      const double vol = space_volume(c);
      c->prof_cr.assign(T.Q, 0.0);
      c->prof_sc.assign(T.Q, 0.0);
      for (int q = 0; q < T.Q; ++q) {
        c->prof_cr[q] = sums[q] / (T.wq[q] * vol);
        c->prof_sc[q] = sums[T.Q + q] / (T.wq[q] * vol);
      }
    }
    c->Rc = 0;
    c->err_c = 0.0;
    c->cap_c = false;
  } else {
    greville_values(c, u, c->grid, s);
    greville_values(c, w, c->grid2, s);
    react_grid(c->grid, c->grid2, c->Cg, c->nunk, c->P.a, c->P.c1, c->P.c2, newton ? 1 : 0, s);
    c->Rc = lowrank(c, c->Cg, c->opt.eps_react, c->Uc_h, c->sc_h, c->Vc, s);
    c->err_c = c->lr_relerr;
    c->cap_c = c->lr_capped;
  }
  rebuild_coefficients(c, s);
}

void residual(st_iga_ctx* c, const double* u, const double* w, double* r, hipStream_t s) {
  ensure_lin(c);
  if (!(c->rfull_u == u && c->rfull_w == w)) quad_pass(c, u, w, true, false, s);
  c->rfull_u = c->rfull_w = nullptr;
  Bufs<double> B = bufs64(c);
  apply_impl<double, double>(c, u, r, c->nt, 0, true, false, B, s);
  axpy(1.0, c->rfull + c->Ns, r, c->nunk, s);
  check_launch();
}

void w_update(st_iga_ctx* c, const double* u, double* w, hipStream_t s) {
  // one pass over u and w: layer 0 of w is the zero row of the matrix
  dense_mode<double, double>(c->DEw.d, c->nt, c->DEw.npad, u, w, 1, c->Ns, s);
  check_launch();
}

std::vector<double> lift_host(st_iga_ctx* c, const st_iga_stimulus* st, int64_t* count) {
  std::vector<double> c0(c->Ns, 0.0);
  int64_t cnt = 0;
  for (int64_t j = 0; j < c->Ns; ++j) {
    double x[3] = {0, 0, 0};
    int64_t r = j;
    for (int l = 0; l < c->d; ++l) {
      x[l] = c->dir[l].grev_x[r % c->n[l]];
      r /= c->n[l];
    }
    bool in = false;
    if (st->u0_kind == 1) in = x[0] < st->u0_center[0];
    else if (st->u0_kind == 2) {
      double r2 = 0.0;
      for (int l = 0; l < c->d; ++l) r2 += (x[l] - st->u0_center[l]) * (x[l] - st->u0_center[l]);
      in = r2 <= st->u0_radius * st->u0_radius;
    }
    if (in) {
      c0[j] = st->u0_value;
      ++cnt;
    }
  }
  if (count) *count = cnt;
  return c0;
}

// Validate the source fields of a stimulus and make them the context's f.
void set_source(st_iga_ctx* c, const st_iga_stimulus* st) {
  Source f;
  if (st->f_kind != 0) {
    if (st->f_kind != 1 && st->f_kind != 2) throw Fail{ST_IGA_EINVAL, "unknown source kind"};
    if (!(st->f_t0 <= st->f_t1)) throw Fail{ST_IGA_EINVAL, "source time window needs f_t0 <= f_t1"};
    if (!std::isfinite(st->f_amp)) throw Fail{ST_IGA_EINVAL, "source amplitude must be finite"};
    if (st->f_kind == 1 && !(st->f_radius > 0)) throw Fail{ST_IGA_EINVAL, "source radius must be positive"};
    if (st->f_kind == 2 && !(st->f_kappa > 0)) throw Fail{ST_IGA_EINVAL, "source kappa must be positive"};
    f.kind = st->f_kind;
    f.d = c->d;
    f.Q1 = c->Q[0];
    for (int l = 0; l < 3; ++l) {
      f.c[l] = st->f_center[l];
      f.v[l] = st->f_kind == 2 ? st->f_velocity[l] : 0.0;
      f.xq[l] = c->xq_dev[l];
    }
    f.r2 = st->f_radius * st->f_radius;
    f.t0 = st->f_t0;
    f.t1 = st->f_t1;
    f.amp = st->f_amp;
    f.kappa = st->f_kappa;
    f.tq = c->tq_dev;
  }
  c->src = f;
  c->rfull_u = c->rfull_w = nullptr;   // a residual cached for the old source is stale
}

template <class F>
st_iga_status guard(st_iga_ctx* c, F&& f) {
  try {
    f();
    return ST_IGA_OK;
  } catch (const Fail& e) {
    if (c) c->err = e.msg;
    return e.st;
  } catch (const std::exception& e) {
    if (c) c->err = e.what();
    return ST_IGA_EINVAL;
  }
}

thread_local std::string g_last_err;

}  // namespace

// =================================================================== C ABI
extern "C" {

void st_iga_default_options(st_iga_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->su = 1;
  o->eps_theta = 0.1;
  o->eps_react = 1e-2;
  o->max_rank = 48;
  o->outer = 0;
  o->alpha = 1.0;
  o->theta_freeze = 1e-4;
  o->tol_nonlin = 1e-10;
  o->tol_lin = 1e-10;
  o->inner_tol = 1e-4;
  o->restart = 30;
  o->max_outer = 60;
  o->max_krylov = 3000;
  o->stall_cycles = 10;
  o->stall_reduction = 1e-3;
  o->picard_switch = 0;
  o->sc_c = 0.1;
  o->precond = 0;
  o->prec = ST_IGA_FP64;
  o->lin_forcing = 0.0;
  o->coef_slab = 0;
  o->reorth = 2;
  o->graphs = 1;
}

size_t st_iga_workspace_bytes(const st_iga_problem* prob, const st_iga_options* opt) {
  st_iga_ctx c;
  try {
    validate(prob, opt);
    c.P = *prob;
    c.opt = *opt;
    host_setup(&c);
    c.ar = Arena();
    plan(&c);
    return c.ar.off + 256;
  } catch (...) {
    return 0;
  }
}

st_iga_status st_iga_setup(const st_iga_problem* prob, const st_iga_options* opt, void* workspace,
                           size_t workspace_bytes, void* stream, st_iga_ctx** out) {
  if (!out) return ST_IGA_EINVAL;
  *out = nullptr;
  std::unique_ptr<st_iga_ctx> c(new st_iga_ctx());
  hipStream_t s = static_cast<hipStream_t>(stream);
  st_iga_status st = guard(c.get(), [&] {
    validate(prob, opt);
    if (!workspace) throw Fail{ST_IGA_EINVAL, "null workspace"};
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) throw Fail{ST_IGA_EINVAL, "workspace must be 256-byte aligned"};
    c->P = *prob;
    c->opt = *opt;
    host_setup(c.get());
    c->ar = Arena();
    plan(c.get());
    const size_t need = c->ar.off;
    if (workspace_bytes < need) throw Fail{ST_IGA_ENOMEM, "workspace too small"};
    c->ar = Arena();
    c->ar.base = static_cast<char*>(workspace);
    c->ar.cap = workspace_bytes;
    c->ar.dry = false;
    plan(c.get());
    upload_all(c.get(), s);
    if (c->banded) {
      // before the first linearization: the shift a c1 of the fast
      // diagonalization as reaction, no theta and no shock capturing
      c->prof_cr.assign(c->dir[c->d].Q, c->P.a * c->P.c1);
      c->prof_sc.clear();
      c->prof_th.clear();
      time_factor(c.get(), s);
    }
    for (int l = 0; l < 4; ++l) c->P.knots[l] = nullptr;
    CK(hipGetDevice(&c->device));
    c->noalloc_ok = noalloc_scratch_init(c->device, c->noalloc_err);
  });
  if (st != ST_IGA_OK) {
    g_last_err = c->err;
    return st;
  }
  *out = c.release();
  return ST_IGA_OK;
}

st_iga_status st_iga_linearize(st_iga_ctx* c, const double* u, const double* w, int32_t refresh_theta, void* stream) {
  if (!c || !u || !w) return ST_IGA_EINVAL;
  return guard(c, [&] {
    if (!c->linearized && c->opt.su == 1 && !refresh_theta) throw Fail{ST_IGA_ESTATE, "theta has never been computed"};
    linearize(c, u, w, refresh_theta != 0, static_cast<hipStream_t>(stream));
    c->rfull_u = c->rfull_w = nullptr;
  });
}

st_iga_status st_iga_set_factors(st_iga_ctx* c, int32_t rt, const double* Ut, const double* st, const double* Vt,
                                 int32_t rc, const double* Uc, const double* sc, const double* Vc) {
  if (!c) return ST_IGA_EINVAL;
  return guard(c, [&] {
    if (rt < 0 || rc < 0 || rt > c->maxR || rc > c->maxR) throw Fail{ST_IGA_EINVAL, "rank out of range"};
    if ((rt > 0 && (!Ut || !st || !Vt)) || (rc > 0 && (!Uc || !sc || !Vc))) throw Fail{ST_IGA_EINVAL, "null factor"};
    hipStream_t s = nullptr;
    c->Rth = rt;
    c->Rc = rc;
    c->Uth_h.assign(Ut, Ut + static_cast<size_t>(c->Nt) * rt);
    c->sth_h.assign(st, st + rt);
    c->Uc_h.assign(Uc, Uc + static_cast<size_t>(c->Nt) * rc);
    c->sc_h.assign(sc, sc + rc);
    if (rt > 0) CK(hipMemcpy(c->Vth, Vt, static_cast<size_t>(c->Ns) * rt * sizeof(double), hipMemcpyHostToDevice));
    if (rc > 0) CK(hipMemcpy(c->Vc, Vc, static_cast<size_t>(c->Ns) * rc * sizeof(double), hipMemcpyHostToDevice));
    rebuild_coefficients(c, s);
  });
}

st_iga_status st_iga_get_factors(st_iga_ctx* c, int32_t* rt, double* Ut, double* st, double* Vt, int32_t* rc,
                                 double* Uc, double* sc, double* Vc) {
  if (!c || !rt || !rc) return ST_IGA_EINVAL;
  return guard(c, [&] {
    *rt = c->Rth;
    *rc = c->Rc;
    if (Ut) std::copy(c->Uth_h.begin(), c->Uth_h.end(), Ut);
    if (st) std::copy(c->sth_h.begin(), c->sth_h.end(), st);
    if (Uc) std::copy(c->Uc_h.begin(), c->Uc_h.end(), Uc);
    if (sc) std::copy(c->sc_h.begin(), c->sc_h.end(), sc);
    if (Vt && c->Rth > 0) CK(hipMemcpy(Vt, c->Vth, static_cast<size_t>(c->Ns) * c->Rth * sizeof(double), hipMemcpyDeviceToHost));
    if (Vc && c->Rc > 0) CK(hipMemcpy(Vc, c->Vc, static_cast<size_t>(c->Ns) * c->Rc * sizeof(double), hipMemcpyDeviceToHost));
  });
}

st_iga_status st_iga_set_stimulus(st_iga_ctx* c, const st_iga_stimulus* stim) {
  if (!c || !stim) return ST_IGA_EINVAL;
  return guard(c, [&] { set_source(c, stim); });
}

st_iga_status st_iga_theta_grid(st_iga_ctx* c, const double* u, const double* w, double* th, void* stream) {
  if (!c || !u || !w || !th) return ST_IGA_EINVAL;
  return guard(c, [&] {
    hipStream_t s = static_cast<hipStream_t>(stream);
    theta_grid(c, u, w, th, s);
    CK(hipStreamSynchronize(s));
  });
}

st_iga_status st_iga_apply(st_iga_ctx* c, const double* x, double* y, void* stream) {
  if (!c || !x || !y) return ST_IGA_EINVAL;
  return guard(c, [&] {
    ensure_lin(c);
    apply64(c, x, y, static_cast<hipStream_t>(stream));
    check_launch();
  });
}

st_iga_status st_iga_precond(st_iga_ctx* c, const double* r, double* z, void* stream) {
  if (!c || !r || !z) return ST_IGA_EINVAL;
  return guard(c, [&] {
    precond64(c, r, z, static_cast<hipStream_t>(stream));
    check_launch();
  });
}

st_iga_status st_iga_precond_noalloc(st_iga_ctx* c, const double* r, double* z, void* stream) {
  if (!c || !r || !z) return ST_IGA_EINVAL;
  return guard(c, [&] {
    if (c->nunk > NOALLOC_MAX_UNKNOWNS)
      throw Fail{ST_IGA_EINVAL, "allocation-free preconditioner: " + std::to_string(c->nunk) +
                                    " unknowns exceed its scratch of " + std::to_string(NOALLOC_MAX_UNKNOWNS)};
    int dev = -1;
    CK(hipGetDevice(&dev));
    if (dev != c->device) throw Fail{ST_IGA_EINVAL, "allocation-free preconditioner: the context's device is not current"};
    double* scr = noalloc_scratch(dev);
    if (!c->noalloc_ok || !scr) throw Fail{ST_IGA_EDEVICE, "allocation-free scratch unavailable: " + c->noalloc_err};
    Bufs<double> B = bufs64(c);
    for (int k = 0; k < NOALLOC_BUFS; ++k) B.t4[k] = scr + static_cast<int64_t>(k) * NOALLOC_MAX_UNKNOWNS;
    B.t4[3] = nullptr;   // not used by the preconditioner
    kprof_suppress(true);
    struct Restore { ~Restore() { kprof_suppress(false); } } restore;
    precond_impl<double, double>(c, r, z, B, static_cast<hipStream_t>(stream));
    check_launch();
  });
}

st_iga_status st_iga_apply_lowp(st_iga_ctx* c, const double* x, double* y, void* stream) {
  if (!c || !x || !y) return ST_IGA_EINVAL;
  return guard(c, [&] {
    ensure_lin(c);
    if (c->opt.prec == ST_IGA_FP64) throw Fail{ST_IGA_EINVAL, "context has no low-precision operators"};
    Op A, Pc;
    if (c->opt.prec == ST_IGA_MIXED_FP32) lowp_ops<float>(c, A, Pc, static_cast<hipStream_t>(stream));
    else lowp_ops<bf16>(c, A, Pc, static_cast<hipStream_t>(stream));
    A(x, y);
    check_launch();
  });
}

st_iga_status st_iga_precond_lowp(st_iga_ctx* c, const double* r, double* z, void* stream) {
  if (!c || !r || !z) return ST_IGA_EINVAL;
  return guard(c, [&] {
    if (c->opt.prec == ST_IGA_FP64) throw Fail{ST_IGA_EINVAL, "context has no low-precision operators"};
    Op A, Pc;
    if (c->opt.prec == ST_IGA_MIXED_FP32) lowp_ops<float>(c, A, Pc, static_cast<hipStream_t>(stream));
    else lowp_ops<bf16>(c, A, Pc, static_cast<hipStream_t>(stream));
    Pc(r, z);
    check_launch();
  });
}

st_iga_status st_iga_residual(st_iga_ctx* c, const double* u, const double* w, double* r, void* stream) {
  if (!c || !u || !w || !r) return ST_IGA_EINVAL;
  return guard(c, [&] {
    hipStream_t s = static_cast<hipStream_t>(stream);
    residual(c, u, w, r, s);
    CK(hipStreamSynchronize(s));
  });
}

st_iga_status st_iga_w_update(st_iga_ctx* c, const double* u, double* w, void* stream) {
  if (!c || !u || !w) return ST_IGA_EINVAL;
  return guard(c, [&] {
    const uintptr_t bytes = static_cast<uintptr_t>(c->nt) * c->Ns * sizeof(double);
    const uintptr_t ua = reinterpret_cast<uintptr_t>(u), wa = reinterpret_cast<uintptr_t>(w);
    if (ua < wa + bytes && wa < ua + bytes) throw Fail{ST_IGA_EINVAL, "u and w overlap"};
    w_update(c, u, w, static_cast<hipStream_t>(stream));
  });
}

st_iga_status st_iga_krylov(st_iga_ctx* c, const double* b, double* x, double tol, int32_t* iters, double* relres,
                            void* stream) {
  if (!c || !b || !x || !(tol > 0)) return ST_IGA_EINVAL;
  int it = 0;
  double rr = 1.0;
  st_iga_status st = guard(c, [&] {
    it = krylov(c, b, x, tol, &rr, static_cast<hipStream_t>(stream));
  });
  if (iters) *iters = it;
  if (relres) *relres = rr;
  return st;
}

st_iga_status st_iga_lift(st_iga_ctx* c, const st_iga_stimulus* stim, double* c0, int64_t* count) {
  if (!c || !stim || !c0) return ST_IGA_EINVAL;
  return guard(c, [&] {
    if (stim->f_kind != 0) throw Fail{ST_IGA_EINVAL, "source terms are not supported"};
    std::vector<double> v = lift_host(c, stim, count);
    std::copy(v.begin(), v.end(), c0);
  });
}

st_iga_status st_iga_solve(st_iga_ctx* c, const st_iga_stimulus* stim, double* u, double* w, st_iga_report* rep,
                           void* stream) {
  if (!c || !stim || !u || !w) return ST_IGA_EINVAL;
  return guard(c, [&] {
    set_source(c, stim);
    hipStream_t s = static_cast<hipStream_t>(stream);
    st_iga_report R;
    std::memset(&R, 0, sizeof(R));
    std::vector<double> c0 = lift_host(c, stim, nullptr);
    for (int k = 0; k < c->nt; ++k)
      CK(hipMemcpyAsync(u + static_cast<int64_t>(k) * c->Ns, c0.data(), c->Ns * sizeof(double), hipMemcpyHostToDevice, s));
    // the fixed-point scheme of Section 3.1 (outer = 2) carries w as a
    // relaxed iterate from w^0 = 0; the other schemes lag w = w(u^k)
    const bool paper_fp = c->opt.outer == 2;
    if (paper_fp) fill(w, 0.0, c->nfull, s);
    CK(hipStreamSynchronize(s));
    bool frozen = false;
    bool converged = false;
    // Newton that keeps growing ||delta||_inf for picard_switch iterations in a
    // row continues as the defect-correction Picard iteration (C_r, alpha =
    // 0.5) for the rest of this solve
    const int32_t outer0 = c->opt.outer;
    const double alpha0 = c->opt.alpha;
    struct RestoreOpt {
      st_iga_ctx* c;
      int32_t o;
      double a;
      ~RestoreOpt() {
        c->opt.outer = o;
        c->opt.alpha = a;
      }
    } restore_opt{c, outer0, alpha0};
    R.switched_at = -1;
    int growth = 0;
    double dprev = -1.0;
    for (int k = 0; k < c->opt.max_outer; ++k) {
      auto t0 = std::chrono::steady_clock::now();
      if (!paper_fp) w_update(c, u, w, s);
      linearize(c, u, w, c->opt.su == 1 && !frozen, s, true);
      residual(c, u, w, c->sol_rhs, s);
      axpby(-1.0, c->sol_rhs, 0.0, c->sol_rhs, c->nunk, s);   // rhs = -N(u)
      CK(hipStreamSynchronize(s));
      auto t1 = std::chrono::steady_clock::now();
      double rr = 1.0;
      // forcing term: with lin_forcing > 0 the k-th linear solve stops at
      // max(tol_lin, min(1e-2, lin_forcing * ||delta_{k-1}||_inf))
      double tol_k = c->opt.tol_lin;
      if (c->opt.lin_forcing > 0.0 && k > 0)
        tol_k = std::max(c->opt.tol_lin, std::min(1e-2, c->opt.lin_forcing * R.delta_inf[std::min(k - 1, ST_IGA_MAX_OUTER_LOG - 1)]));
      const int it = krylov(c, c->sol_rhs, c->sol_dx, tol_k, &rr, s);
      if (paper_fp) {
        // w~ from L w~ = G(u^k), then w^{k+1} = alpha w~ + (1 - alpha) w^k
        // (t4[3] is free once the linear solve has finished)
        w_update(c, u, c->t4[3], s);
        axpby(c->opt.alpha, c->t4[3], 1.0 - c->opt.alpha, w, c->nfull, s);
      }
      add_unknowns(u, c->sol_dx, c->opt.alpha, c->nunk, c->Ns, s);
      const double dinf = c->opt.alpha * dev_absmax(c, c->sol_dx, c->nunk, s);
      auto t2 = std::chrono::steady_clock::now();
      R.seconds_linearize += std::chrono::duration<double>(t1 - t0).count();
      R.seconds_krylov += std::chrono::duration<double>(t2 - t1).count();
      if (k < ST_IGA_MAX_OUTER_LOG) {
        R.krylov[k] = it;
        R.rank_theta[k] = c->Rth;
        R.rank_react[k] = c->Rc;
        R.delta_inf[k] = dinf;
        R.lin_relres[k] = rr;
        R.lr_relerr_theta[k] = c->err_th;
        R.lr_relerr_react[k] = c->err_c;
      }
      R.rank_capped += (c->cap_th ? 1 : 0) + (c->cap_c ? 1 : 0);
      R.krylov_total += it;
      R.outer_iters = k + 1;
      R.final_delta_inf = dinf;
      if (outer0 == 0 && c->opt.picard_switch > 0 && R.switched_at < 0) {
        growth = (dprev >= 0.0 && dinf > dprev) ? growth + 1 : 0;
        if (growth >= c->opt.picard_switch) {
          c->opt.outer = 1;
          c->opt.alpha = 0.5;
          R.switched_at = k + 1;
        }
      }
      dprev = dinf;
      if (dinf <= c->opt.theta_freeze) frozen = true;
      if (dinf <= c->opt.tol_nonlin) {
        converged = true;
        break;
      }
    }
    if (!paper_fp) w_update(c, u, w, s);
    CK(hipStreamSynchronize(s));
    if (rep) *rep = R;
    if (!converged) throw Fail{ST_IGA_ENOCONV, "outer iteration limit reached"};
  });
}

st_iga_status st_iga_newton_step(st_iga_ctx* c, const double* u_in, double* u_out, double* w, int32_t refresh_theta,
                                 double tol, int32_t* iters, double* relres, double* delta_inf, void* stream) {
  if (!c || !u_in || !u_out || !w || !(tol > 0)) return ST_IGA_EINVAL;
  return guard(c, [&] {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (u_out != u_in) CK(hipMemcpyAsync(u_out, u_in, c->nfull * sizeof(double), hipMemcpyDeviceToDevice, s));
    w_update(c, u_out, w, s);
    if (!c->linearized && c->opt.su == 1 && !refresh_theta) throw Fail{ST_IGA_ESTATE, "theta has never been computed"};
    linearize(c, u_out, w, refresh_theta != 0, s, true);
    residual(c, u_out, w, c->sol_rhs, s);
    axpby(-1.0, c->sol_rhs, 0.0, c->sol_rhs, c->nunk, s);
    double rr = 1.0;
    const int it = krylov(c, c->sol_rhs, c->sol_dx, tol, &rr, s);
    add_unknowns(u_out, c->sol_dx, c->opt.alpha, c->nunk, c->Ns, s);
    const double dinf = c->opt.alpha * dev_absmax(c, c->sol_dx, c->nunk, s);
    if (iters) *iters = it;
    if (relres) *relres = rr;
    if (delta_inf) *delta_inf = dinf;
  });
}

st_iga_status st_iga_profile(st_iga_ctx* c, int32_t enable) {
  if (!c) return ST_IGA_EINVAL;
  kprof_enable(enable != 0);
  return ST_IGA_OK;
}

st_iga_status st_iga_profile_read(st_iga_ctx* c, int32_t cls, double* ms, int64_t* launches, double* bytes,
                                  double* flops, int32_t reset) {
  if (!c || cls < 0 || (cls >= K_NCLASS && (cls < 100 || cls >= 196))) return ST_IGA_EINVAL;
  return guard(c, [&] { kprof_read(cls, ms, launches, bytes, flops, reset); });
}

st_iga_status st_iga_profile_record(st_iga_ctx* c, int64_t i, int32_t* fn, double* ms, double* bytes,
                                    double* flops) {
  if (!c) return ST_IGA_EINVAL;
  int f = 0;
  if (!kprof_record(i, &f, ms, bytes, flops)) return ST_IGA_EINVAL;
  if (fn) *fn = f;
  return ST_IGA_OK;
}

st_iga_status st_iga_sizes(const st_iga_ctx* c, int64_t* o) {
  if (!c || !o) return ST_IGA_EINVAL;
  o[0] = c->d;
  o[1] = c->n[0];
  o[2] = c->n[1];
  o[3] = c->n[2];
  o[4] = c->nt;
  o[5] = c->Ns;
  o[6] = c->Nt;
  o[7] = c->nunk & 0xffffffffLL;
  o[8] = c->nunk >> 32;
  return ST_IGA_OK;
}

st_iga_status st_iga_destroy(st_iga_ctx* c) {
  delete c;
  return ST_IGA_OK;
}

const char* st_iga_last_error(const st_iga_ctx* c) { return c ? c->err.c_str() : g_last_err.c_str(); }

st_iga_status st_iga_host_symeig(int32_t n, const double* A, double* Q, double* lam) {
  if (n < 1 || !A || !Q || !lam) return ST_IGA_EINVAL;
  st_iga_ctx c;
  return guard(&c, [&] {
    std::vector<double> M(A, A + static_cast<size_t>(n) * n), U, l;
    std::string err;
    if (!sym_eig(M, n, U, l, err)) throw Fail{ST_IGA_ENOCONV, err};
    std::copy(U.begin(), U.end(), Q);
    std::copy(l.begin(), l.end(), lam);
  });
}

st_iga_status st_iga_host_query(const st_iga_problem* prob, int32_t what, int32_t dir, double* out, int64_t cap,
                                int64_t* len) {
  st_iga_ctx c;
  st_iga_options o;
  st_iga_default_options(&o);
  return guard(&c, [&] {
    validate(prob, &o);
    c.P = *prob;
    c.opt = o;
    host_setup(&c);
    if (dir < 0 || dir > c.d) throw Fail{ST_IGA_EINVAL, "bad direction"};
    const Dir1D& D = c.dir[dir];
    std::vector<double> v;
    switch (what) {
      case 0: v = D.grev_x; break;
      case 1: v = gram1d(D, 0, 0, nullptr); break;
      case 2: v = gram1d(D, 1, 1, nullptr); break;
      case 3: v = gram1d(D, 0, 1, nullptr); break;
      case 4: v = c.tauq; break;
      case 5: if (dir == c.d) throw Fail{ST_IGA_EINVAL, "spatial only"}; v = c.lam_h[dir]; break;
      case 6: if (dir == c.d) throw Fail{ST_IGA_EINVAL, "spatial only"}; v = c.Us_h[dir]; break;
      case 7: {
        v = c.fd.U;
        v.insert(v.end(), c.fd.mu.begin(), c.fd.mu.end());
        v.insert(v.end(), c.fd.l.begin(), c.fd.l.end());
        v.push_back(c.fd.sigma);
        break;
      }
      case 8: v = D.xq; v.insert(v.end(), D.wq.begin(), D.wq.end()); break;
      case 9: for (int f : D.first) v.push_back(f); break;
      case 10: {
        std::vector<int> e0, e1;
        support_windows(D, dir == c.d ? 1 : 0, e0, e1);
        for (size_t i = 0; i < e0.size(); ++i) { v.push_back(e0[i]); v.push_back(e1[i]); }
        break;
      }
      case 11: {
        v = {c.cf ? 1.0 : 0.0, static_cast<double>(c.cf_slab), static_cast<double>(c.cf_nchunk)};
        for (int x : c.cf_chunks_h) v.push_back(x);
        break;
      }
      default: throw Fail{ST_IGA_EINVAL, "unknown query"};
    }
    if (len) *len = static_cast<int64_t>(v.size());
    if (out) std::copy(v.begin(), v.begin() + std::min<int64_t>(cap, v.size()), out);
  });
}

}  // extern "C"
