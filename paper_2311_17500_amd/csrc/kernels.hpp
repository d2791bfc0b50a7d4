// Launch wrappers of the gfx950 kernels (implemented in kernels.hip).
//
// Array views: a tensor is addressed as [outer][n][inner] around the axis a
// kernel acts on (inner = product of the faster axes, outer = product of the
// slower ones).  All index arithmetic is 64-bit.
#pragma once
#include <hip/hip_runtime_api.h>
#include <hip/hip_bf16.h>
#include <cstdint>
#include <string>

namespace stiga {

typedef __hip_bfloat16 bf16;

// Source term f(x, t) of eq. (3.1) at the space-time Gauss points: kind 1 is
// amp on the closed ball |x - c| <= r during [t0, t1], kind 2 the moving
// Gaussian amp exp(-kappa |x - c - v t|^2) during [t0, t1] (the two stimuli of
// the paper's experiments); kind 0 is f = 0.  xq / tq are the Gauss abscissae
// of each spatial direction and of time (device arrays).
struct Source {
  int kind = 0, d = 0;
  int Q1 = 1;                 // Gauss points along x_1 (column decomposition of the fused pass)
  double c[3] = {0.0, 0.0, 0.0}, v[3] = {0.0, 0.0, 0.0};
  double r2 = 0.0, t0 = 0.0, t1 = 0.0, amp = 0.0, kappa = 0.0;
  const double* xq[3] = {nullptr, nullptr, nullptr};
  const double* tq = nullptr;
};

// Kernel classes for the optional HIP-event profiler (host-side timing of
// individual launches on the stream they run on).
enum KClass { K_GATHER = 0, K_TIME_MIX, K_ARROW, K_MULTIDOT, K_UPDATE, K_POINTWISE, K_MAX, K_BANDED, K_EXPAND,
              K_DENSE, K_COEF, K_NCLASS };
void kprof_enable(bool on);
// while on (per thread), launches record no profiler events (no event creation)
void kprof_suppress(bool on);
bool kprof_enabled();
// class recorded for gather launches until changed (K_GATHER by default)
void kprof_gather_class(int cls);
// Sum of launch durations (ms), launch count and algorithmic bytes of a class since the last reset;
// synchronizes the recorded events.  Resets when reset != 0.
void kprof_read(int cls, double* ms, int64_t* launches, double* bytes, double* flops, int reset);
// Launch i since the last reset (function id, duration, bytes, flops); false past the end.
bool kprof_record(int64_t i, int* fn, double* ms, double* bytes, double* flops);

// Device view of a gather table: y[i] = sum_w coef[i*W+w] * x[col[i*W+w] - in_base],
// terms with the input index outside [0, n_in) skipped.
template <class C>
struct DTable {
  const int* col = nullptr;
  const C* coef = nullptr;
  const int* c0 = nullptr;   // contiguous window starts (see make_contiguous), or null
  int n_out = 0, W = 0;
};

// y[o][i][k] = alpha * sum_w coef * x[o][col-in_base][k] + beta * y[o][i][k]
// (beta == 0: y is not read).  Input element type Ti, output To, arithmetic C.
template <class Ti, class To, class C>
void gather(const DTable<C>& t, const Ti* x, To* y, int64_t outer, int64_t inner, int n_in, int in_base,
            C alpha, C beta, hipStream_t s);

// Same, restricted to output rows [r0, r0 + nr) of the table (y holds only those rows).
template <class Ti, class To, class C>
void gather_rows(const DTable<C>& t, int r0, int nr, const Ti* x, To* y, int64_t outer, int64_t inner, int n_in,
                 int in_base, C alpha, C beta, hipStream_t s);

// Two tables with the same contiguous windows (P.c0) along one axis in one
// pass: out1 = P x (skipped when out1 is null), out2 = alpha Q x + beta P z.
// Returns false (nothing launched) when the tables do not qualify (no
// windows, different widths, W not in {2,3,4,5,7,9,11}, inner < 2).
template <class S, class C>
bool gather_dual(const DTable<C>& P, const DTable<C>& Q, const S* x, const S* z, S* out1, S* out2, int64_t outer,
                 int64_t inner, int n_in, int in_base, C alpha, C beta, hipStream_t s);

// y[o][i][k] = max_{w < cnt[i]} x[o][start[i]+w][k]
void mode_max(const int* start, const int* cnt, int n_out, const double* x, double* y, int64_t outer,
              int64_t inner, int n_in, hipStream_t s);

// Coefficient part of the operator at the spatial Gauss points, rows t in [t0, t1):
//   out[t - t0][q] = sum_{r in [r0,r1)} Psi[r][q] sum_w T[r][t][w] * Z[t+1-p+w - in_base][q]
// (T has Nt rows per rank, at least t1; inputs outside [0, n_in) skipped).
template <class S, class C>
void time_mix(const C* T, const S* Psi, int r0, int r1, int Nt, int t0, int t1, int p, const S* Z, int n_in,
              int in_base, S* out, int64_t Qs, hipStream_t s);

// Reaction term with a coefficient given at every space-time Gauss point
// (Cq [Q_t][Qs], Gauss weights included), over output rows [t0, t1) of the
// unknowns: out[t - t0][q] = beta out + sum over the time Gauss points g in
// supp b_{t+1} of Bv(g, t+1) Cq[g][q] (sum_a B(g, a) Z[a][q])
//            + B'(g, t+1) Rq[g][q] (sum_a B'(g, a) Z[a][q]).
// Z holds the spatially expanded input layers of full indices [lo_full,
// lo_full + nl).  Bt: time basis values at the Gauss points (contiguous
// windows, W = p + 1); Bv: test values in the same layout (null: Bt); Bd:
// time derivatives in the same layout (read only with Rq); Cq or Rq null:
// that term is skipped; re0/re1: per full time row, the range of time
// elements in its support.
template <class S, class C>
void react_point(const S* Z, int nl, int lo_full, const DTable<C>& Bt, const C* Bv, const C* Bd, const int* re0,
                 const int* re1, const C* Cq, const C* Rq, int64_t Qs, int t0, int t1, int p, S* out, C beta,
                 hipStream_t s);

// Banded time solves of the SUPG preconditioner: per spatial mode j the
// matrix T_j = A + (lam[j] - shift) B (bands [t][2p+1] of X_t, column t-p+k)
// factorized without pivoting into F ([t][2p+1][Ns]: multipliers, reciprocal
// pivot, upper entries); band_solve applies T_j^{-1} to r ([t][Ns]) into x
// (no aliasing).  False (nothing launched) for p outside 1..5.
bool band_factor(const double* A, const double* B, int Nt, const double* lam, double shift, int64_t Ns, int p,
                 double* F, hipStream_t s);
template <class S, class C>
bool band_solve(const C* F, int Nt, int64_t Ns, int p, const S* r, S* x, hipStream_t s);
// out[g] = sum of the Qs values of row g of X ([rows][Qs]).
void row_sums(const double* X, int rows, int64_t Qs, double* out, hipStream_t s);

// Coefficient part along the slowest spatial axis in one kernel (time_mix
// between the expansion to that axis' Gauss points and the projection back):
//   out[t - t0][i][c] = sum_{q in axis Gauss points} Bl[q][i - efirst(q)] *
//                       sum_{r in [r0,r1)} Psi[r][q*Qin + c] sum_w T[r][t][w] z[t+1-p+w - in_base][q][c],
//   z[j][q][c] = sum_k Bl[q][k] Z[j][efirst(q)+k][c],
// T: [rank][Nt][2 p_t + 1] with Nt >= t1 + 7 rows per rank (rows past the
// last time row zero; a thread reads 8 rows from its first),
// Z: [n_in][nd][Qin], out: [t1-t0][nd][Qin], Bl: [Q][ps+1] basis values at the
// axis' Gauss points (element-major, ps+1 points per element), efirst: first
// B-spline of each element, chunks: nchunk x {e0, e1, d0, d1} (elements
// walked and B-splines stored by one thread).  Returns false (nothing
// launched) for degrees outside p_t <= 5, p_s <= 4.
template <class S, class C>
bool coef_fused(const C* T, const S* Psi, int r0, int r1, int Nt, int t0, int t1, int pt, int ps, const S* Z,
                int n_in, int in_base, const C* Bl, const int* efirst, const int* chunks, int nchunk, int nd,
                int64_t Qin, S* out, int64_t Qs, hipStream_t s);

// Quadrature pass fused along the slowest spatial axis (FP64), see
// k_quad_fused: inputs [ne*nqt][nd][Qin] expanded along the faster axes
// (d = 3: A0 = B0 B0 u, A1 = B0 B2 u (x1 value, x2 second derivative),
// A2 = B2 B0 u; d = 2: A0 = B0 u, A2 = B2 u, A1 unused), UT and WW the
// value expansions of u_t and w; B0, B2: [Q][ps+1] basis values and second
// derivatives at the axis' Gauss points; wt: time weights of the ne*nqt
// rows; win: products of the faster axes' Gauss weights [Qin]; wd: Gauss
// weights of the axis [Q].  Outputs (each optional): G [ne*nqt][nd][Qin]
// (weighted ionic current projected onto the axis' B-splines), M
// [ne][nel_d][Qin] (element maxima of |R| over the axis and time), Cq and
// Rq (omega C_r and omega |R| at every space-time Gauss point, layout
// [q0 + row][Qs]), and block
// maxima of |u|, |u_t| at part[2(boff + b)], part[2(boff + b) + 1].  Returns
// the number of blocks written (or -1 if the degrees are not supported:
// d in {2, 3}, ps <= 4, nqt <= 6).  With e0x2 given (d = 3), A0 = B0 u and
// A2 = B2 u along x1, UT and WW are expanded along x1 only ([ne*nqt][nd][n2]
// [Q1], A1 unused) and the kernel forms the x2 expansion: rows f2x[q2] + k
// (k <= ps, all < n2) with values e0x2 and second derivatives e2x2
// ([Q2][ps+1]) at x2 Gauss point q2 = c / Q1.
int64_t quad_fused(int d, int ps, int nqt, const double* A0, const double* A1, const double* A2, const double* UT,
                   const double* WW, int nd, int64_t Qin, int ne, const double* B0, const double* B2,
                   const int* efirst, const int* chunks, int nchunk, const double* wt, const double* win,
                   const double* wd, double sL,
                   double sM, double sF, double Cm, double a, double c1, double c2, double* G, double* M, int nel_d,
                   double* part, int64_t boff, hipStream_t s, int n2, int Q1, const double* e0x2,
                   const double* e2x2, const int* f2x, const Source& f, int q0, double* Cq, double* Rq,
                   int64_t Qs);

// Dense mode product on MFMA: y[o][i][k] = sum_j A[i][j] x[o][j][k], A given
// zero-padded as npad x npad (npad = 16 * ceil(n / 16) <= 144), row-major.
template <class S, class C>
void dense_mode(const C* Ap, int n, int npad, const S* x, S* y, int64_t outer, int64_t inner, hipStream_t s);
// The same product with BF16 operands on the BF16 MFMA (FP32 accumulation):
// Ab is the zero-padded BF16 copy of the matrix.  Returns false (nothing
// launched) when the layout is not supported (odd inner, npad > 144); the
// caller then uses dense_mode<bf16, float>.
bool dense_mode_b16(const bf16* Ab, int n, int npad, const bf16* x, bf16* y, int64_t outer, int64_t inner,
                    hipStream_t s);

// Arrowhead solve of the fast-diagonalization core, one spatial mode per thread:
// the first np time-mode pairs are 2x2 blocks (values mu), the remaining
// N_t - 1 - 2 np modes 1x1 zero blocks, the last mode the arrow (l, sigma).
template <class S, class C>
void arrowhead(const S* r, S* y, const C* lam, const C* mu, int np, const C* l, C sigma, C Cm,
               int Nt, int64_t Ns, hipStream_t s);

// Deterministic reductions (two stages, fixed order).
// Time part of the FD preconditioner in one pass (FP32 arithmetic): z[., j]
// = U_t core_j^{-1} U_t^T x[., j] for every spatial mode j < Ns, with the
// arrowhead core of arrowhead() (same lam, mu, l, np, sigma, Cm).  UtT, Ut:
// padded npad x npad FP32 matrices; x, z: [Nt][Ns].  Returns false (nothing
// launched) unless npad is 16, 32, 48 or 64 and Nt <= npad.
template <class S>
bool time_core(const float* UtT, const float* Ut, int Nt, int npad, const S* x, S* z, int64_t Ns, const float* lam,
               const float* mu, int np, const float* l, float sigma, float Cm, hipStream_t s);

int reduce_blocks(int64_t n);
// part[b*k + j] = partial of <V_j, w> over block b; V_j = V + j*ldv (T: basis storage, FP64 accumulation)
template <class T>
void multidot_partial(const T* V, int64_t ldv, int k, const T* w, int64_t n, double* part, int nb, hipStream_t s);
// out[j] = sum_b part[b*k + j]
// Partial sums of V_i . a and V_i . b for i < k in one pass over V:
// part[b][2k] = {V_i . a ..., V_i . b ...}; finalize_sum with 2k values.
template <class T>
void multidot2_partial(const T* V, int64_t ldv, int k, const T* a, const T* b, int64_t n, double* part, int nb,
                       hipStream_t s);
// Delayed second Gram-Schmidt pass (columns j, j + 1 of V hold u and w, dots
// the 2(j + 1) finalized sums of multidot2 over the first j + 1 columns):
// column j <- (u - sum_{i<j} s_i V_i) / alpha, column j + 1 <- (w - sum_{i<j}
// t_i V_i - h v) / alpha, partial |w'|^2 into part, {alpha, h} into sc[0], sc[1].
template <class T>
void dcgs_update_partial(T* V, int64_t ldv, int j, const double* dots, int64_t n, double* part, int nb, double* sc,
                         hipStream_t s);
void finalize_sum(const double* part, int nb, int k, double* out, hipStream_t s);

// Givens state of one FGMRES(m) cycle on the device (FP64, offsets in doubles):
// the raw and the rotated Hessenberg matrices Hr and R ((m+1) x m, row-major),
// the rotations cs, sn (m), the rotated right-hand side g and its provisional
// entries gpre (m+1), the previous step's alpha, per step parity a copy of
// the provisional column of R and of g at its diagonal, and per step parity
// the values the host reads: alpha, h, beta, g[j] after column j-1 is
// completed, g[j+1] after the provisional rotation of column j, and a flag
// (1: non-finite coefficients, 2: zero start vector).
struct GivensLayout {
  int64_t Hr, R, cs, sn, g, gpre, ap, snapR, snapg, out, total;
};
inline GivensLayout givens_layout(int m) {
  GivensLayout L;
  const int64_t hm = static_cast<int64_t>(m + 1) * m;
  L.Hr = 0;
  L.R = L.Hr + hm;
  L.cs = L.R + hm;
  L.sn = L.cs + m;
  L.g = L.sn + m;
  L.gpre = L.g + m + 1;
  L.ap = L.gpre + m + 1;
  L.snapR = L.ap + 1;
  L.snapg = L.snapR + 2 * (m + 1);
  L.out = L.snapg + 2;
  L.total = L.out + 2 * 8;
  return L;
}
// Arnoldi step j of the FGMRES cycle with the delayed second Gram-Schmidt
// pass: D[256] = |w'|^2 = sum of the nb partials, then from the step's
// scalars D (dots of u at [0, j), of w at [j+1, 2j+1), alpha at 128, h at
// 129) completes Hessenberg column j - 1, sets the provisional column j and
// applies the Givens rotations (one block; m <= 64).
void norm_givens(const double* part, int nb, double* D, double* G, const GivensLayout& L, int m, int j,
                 hipStream_t s);
// y[0..jn) = R^{-1} g by back substitution; column snap_j (if >= 0) and g at
// its diagonal come from that step's copies (a later step may have run).
void givens_solve(const double* G, const GivensLayout& L, int m, int jn, int snap_j, double* y, hipStream_t s);
// w -= sum_j h[j] V_j ; part[b] = partial ||w||^2 (h read from device)
template <class T>
void update_norm_partial(const T* V, int64_t ldv, int k, const double* h, T* w, int64_t n, double* part, int nb,
                         hipStream_t s);
// part[b] = partial max |x| (kind 0) or sum x^2 (kind 1)
void absmax_partial(const double* x, int64_t n, double* part, int nb, hipStream_t s);
void sumsq_partial(const double* x, int64_t n, double* part, int nb, hipStream_t s);
void finalize_max(const double* part, int nb, double* out, hipStream_t s);
// out[q] = max_b part[2 b + q] for q = 0, 1 (interleaved pairs of nb blocks)
void finalize_max2(const double* part, int64_t nb, double* out, hipStream_t s);

// x = a * x (scale from a device scalar: x *= 1/sqrt(*nrm2) if inv_sqrt)
template <class T>
void scale_by_dev(T* x, int64_t n, const double* nrm2, hipStream_t s);
template <class T>
void scale_to(const double* x, double a, T* y, int64_t n, hipStream_t s);      // y = a x
template <class T>
void sub_from(const double* b, const T* y, double* r, int64_t n, hipStream_t s);  // r = b - y
void axpy(double a, const double* x, double* y, int64_t n, hipStream_t s);            // y += a x
void axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s);  // y = a x + b y
// x += sum_j c[j] Z_j (c on device)
template <class T>
void combine(const T* Z, int64_t ldz, int k, const double* c, double* x, int64_t n, hipStream_t s);
template <class A, class B>
void convert(const A* x, B* y, int64_t n, hipStream_t s);
void fill(double* x, double v, int64_t n, hipStream_t s);

// Pointwise linearization at space-time Gauss points of one time chunk:
//   g = omega * I_ion(u, w);  absR = |Cm ut - lap + I_ion(u, w)|;
//   part[2b] = max |u|, part[2b+1] = max |ut| over block b.
void pointwise_ionic(const double* u, const double* ut, const double* lap, const double* w,
                     const double* wt_time, const double* wt_space, int64_t Qs, int nq_t, double Cm,
                     double a, double c1, double c2, double* g, double* absR, double* part, int nb,
                     hipStream_t s,
                     const Source& f, int q0, int Q1, int Q2, double* Cq, double* Rq);
// R[g][q] *= fac[g] / (Cm (maxes[0] invT + maxes[1])), 0 where that is 0
// (n = Q_t Qs values, Gauss-point layout [g][q]).
void sc_scale(double* R, const double* fac, const double* maxes, double Cm, double invT, int64_t Qs, int64_t n,
              hipStream_t s);
// theta = min(num/den, 1) with den from device maxima (den = Cm (umax/T + utmax)); den == 0 -> num > 0
void theta_finish(double* th, int64_t n, const double* maxes, double Cm, double invT, hipStream_t s);
// coefficient grid: newton ? dI/du : C_r at (u, w)
void react_grid(const double* u, const double* w, double* c, int64_t n, double a, double c1, double c2, int newton,
                hipStream_t s);
// Gram matrix G = C C^T of an (m x n) row-major matrix (partials per block, then reduce)
void gram_partial(const double* C, int m, int64_t n, double* part, int nb, hipStream_t s);
// V[j][r] = sum_i C[i][j] U[i][r] * inv_s[r]  (U: m x R row-major on device)
void right_factor(const double* C, int m, int64_t n, const double* U, const double* inv_s, int R, double* V,
                  hipStream_t s);
// Psi[r][q] *= wq[q] (spatial weights, length Qs) for r in [0, R)
void scale_rows(double* Psi, int R, int64_t Qs, const double* wq, hipStream_t s);
// out[r][j] = V[j][r] (transpose N x R -> R x N)
void transpose_nr(const double* V, int64_t N, int R, double* out, hipStream_t s);
// Newton update u[layers 1..] += alpha * delta; returns nothing (norm via absmax)
void add_unknowns(double* u_full, const double* delta, double alpha, int64_t n_unk, int64_t Ns, hipStream_t s);

// Allocation-free entry points: NOALLOC_BUFS intermediate vectors of at most
// NOALLOC_MAX_UNKNOWNS FP64 entries in a static device array per GPU.
constexpr int NOALLOC_BUFS = 3;
constexpr int64_t NOALLOC_MAX_UNKNOWNS = int64_t(1) << 21;
// Resolve (once per device; the device must be current) and keep the address
// of that device's copy of the array; false with a message on failure.
bool noalloc_scratch_init(int device, std::string& err);
// The resolved address for `device` (null if never resolved).
double* noalloc_scratch(int device);

}  // namespace stiga
