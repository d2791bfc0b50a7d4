// gfx950 kernels of the space-time isogeometric solver.
//
// Design notes (CDNA4: 64-wide wavefronts, 256 CUs in 8 XCDs, HBM3E):
//  * Every 1D operator (banded Galerkin matrices, B-spline evaluation at
//    Gauss points, their transposes, hat interpolation, dense eigenvector
//    blocks) is a row table (col, coef) applied along one tensor axis.  The
//    thread owning output (o, i, k) reads x[o][col][k]; consecutive lanes take
//    consecutive k (or consecutive i on the fastest axis), so loads are
//    coalesced and the 2p+1 overlapping rows are served from L1/L2.
//  * The coefficient part of the operator runs one thread per spatial Gauss
//    point sweeping all time rows with a (2p+1)-wide register window.
//  * Reductions are two-stage with a fixed summation order, so results are
//    bitwise reproducible run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "kernels.hpp"

namespace stiga {

namespace {

constexpr int TPB = 256;

__device__ __forceinline__ double to_c(double v, double) { return v; }
__device__ __forceinline__ float to_c(float v, float) { return v; }
__device__ __forceinline__ double to_c(float v, double) { return static_cast<double>(v); }
__device__ __forceinline__ float to_c(double v, float) { return static_cast<float>(v); }
__device__ __forceinline__ float to_c(bf16 v, float) { return __bfloat162float(v); }
__device__ __forceinline__ double to_c(bf16 v, double) { return static_cast<double>(__bfloat162float(v)); }

template <class T>
__device__ __forceinline__ T from_c(double v);
template <class T>
__device__ __forceinline__ T from_c(float v);
template <>
__device__ __forceinline__ double from_c<double>(double v) { return v; }
template <>
__device__ __forceinline__ float from_c<float>(double v) { return static_cast<float>(v); }
template <>
__device__ __forceinline__ float from_c<float>(float v) { return v; }
template <>
__device__ __forceinline__ double from_c<double>(float v) { return static_cast<double>(v); }
template <>
__device__ __forceinline__ bf16 from_c<bf16>(float v) { return __float2bfloat16(v); }
template <>
__device__ __forceinline__ bf16 from_c<bf16>(double v) { return __float2bfloat16(static_cast<float>(v)); }

inline unsigned grid_for(int64_t n, int tpb = TPB) { return static_cast<unsigned>((n + tpb - 1) / tpb); }

// ---------------------------------------------------------------- profiler
// Process-wide profiler; enabling it is meant for one solver thread at a time
// (benchmarks).  The gather tag is per thread so concurrent contexts never race.
thread_local int t_gather_cls = 0;
thread_local bool t_prof_suppress = false;   // no events recorded (allocation-free entry points)
struct ProfState {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec {
    int cls;   // purpose class
    int fn;    // kernel function id + 32 * precision (0 f64, 1 f32, 2 bf16)
    hipEvent_t a, b;
    double bytes, flops;
  };
  std::vector<Rec> rec;
};
ProfState& prof() {
  static ProfState p;
  return p;
}
hipEvent_t prof_event() {
  ProfState& p = prof();
  if (p.used == p.pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    p.pool.push_back(e);
  }
  return p.pool[p.used++];
}
// RAII bracket around one launch
template <class S> constexpr int prec_code() { return std::is_same<S, double>::value ? 0 : (std::is_same<S, float>::value ? 1 : 2); }
struct ProfScope {
  int cls, fn;
  hipStream_t s;
  hipEvent_t a = nullptr;
  double bytes, flops;
  ProfScope(int c, int f, hipStream_t st, double by, double fl = 0.0) : cls(c), fn(f), s(st), bytes(by), flops(fl) {
    if (prof().on && !t_prof_suppress) {
      a = prof_event();
      if (a) hipEventRecord(a, s);
    }
  }
  ~ProfScope() {
    if (a) {
      hipEvent_t b = prof_event();
      if (b) {
        hipEventRecord(b, s);
        prof().rec.push_back({cls, fn, a, b, bytes, flops});
      }
    }
  }
};

// ---------------------------------------------------------------- gather
template <class Ti, class To, class C, class I>
__global__ void __launch_bounds__(TPB) k_gather(const int* __restrict__ col, const C* __restrict__ coef, int W,
                                                int n_out, const Ti* __restrict__ x, To* __restrict__ y,
                                                I inner, int n_in, int in_base, C alpha, C beta, I total) {
  const I idx = static_cast<I>(blockIdx.x) * static_cast<I>(blockDim.x) + static_cast<I>(threadIdx.x);
  if (idx >= total) return;
  const I k = idx % inner;
  const I t = idx / inner;
  const int i = static_cast<int>(t % static_cast<I>(n_out));
  const I o = t / static_cast<I>(n_out);
  const int* cr = col + static_cast<int64_t>(i) * W;
  const C* cf = coef + static_cast<int64_t>(i) * W;
  const Ti* xb = x + static_cast<int64_t>(o) * n_in * static_cast<int64_t>(inner) + k;
  C acc = C(0);
  for (int w = 0; w < W; ++w) {
    const int c = cr[w] - in_base;
    if (static_cast<unsigned>(c) < static_cast<unsigned>(n_in))
      acc += cf[w] * to_c(xb[static_cast<int64_t>(c) * static_cast<int64_t>(inner)], C(0));
  }
  C r = alpha * acc;
  if (beta != C(0)) r += beta * to_c(y[idx], C(0));
  y[idx] = from_c<To>(r);
}


// Vectorized variant for inner % 4 == 0: each thread produces 4 consecutive k
// of one output row.  Threads of a block share one row block (o, i) when
// inner >= 4 * blockDim, so the table row is read once per wave.
template <class T> struct V4;
template <> struct V4<double> { typedef double4 T; };
template <> struct V4<float> { typedef float4 T; };

template <class S, class C>
__device__ __forceinline__ void load4(const S* p, C* v) {
  typedef typename V4<S>::T T4;
  const T4 t = *reinterpret_cast<const T4*>(p);
  v[0] = static_cast<C>(t.x); v[1] = static_cast<C>(t.y); v[2] = static_cast<C>(t.z); v[3] = static_cast<C>(t.w);
}
template <>
__device__ __forceinline__ void load4<bf16, float>(const bf16* p, float* v) {
  for (int e = 0; e < 4; ++e) v[e] = __bfloat162float(p[e]);
}
template <class S, class C>
__device__ __forceinline__ void store4(S* p, const C* v) {
  typedef typename V4<S>::T T4;
  T4 t;
  t.x = static_cast<S>(v[0]); t.y = static_cast<S>(v[1]); t.z = static_cast<S>(v[2]); t.w = static_cast<S>(v[3]);
  *reinterpret_cast<T4*>(p) = t;
}
template <>
__device__ __forceinline__ void store4<bf16, float>(bf16* p, const float* v) {
  for (int e = 0; e < 4; ++e) p[e] = __float2bfloat16(v[e]);
}


template <int VEC, class S, class C>
__device__ __forceinline__ void loadv(const S* p, C* v) {
  if constexpr (VEC == 4) {
    load4<S, C>(p, v);
  } else if constexpr (VEC == 1) {
    v[0] = to_c(p[0], C(0));
  } else {
    if constexpr (std::is_same<S, bf16>::value) {
      v[0] = __bfloat162float(p[0]); v[1] = __bfloat162float(p[1]);
    } else {
      typedef typename std::conditional<std::is_same<S, double>::value, double2, float2>::type T2;
      const T2 t = *reinterpret_cast<const T2*>(p);
      v[0] = static_cast<C>(t.x); v[1] = static_cast<C>(t.y);
    }
  }
}
template <int VEC, class S, class C>
__device__ __forceinline__ void storev(S* p, const C* v) {
  if constexpr (VEC == 4) {
    store4<S, C>(p, v);
  } else if constexpr (VEC == 1) {
    p[0] = from_c<S>(v[0]);
  } else {
    if constexpr (std::is_same<S, bf16>::value) {
      p[0] = __float2bfloat16(v[0]); p[1] = __float2bfloat16(v[1]);
    } else {
      typedef typename std::conditional<std::is_same<S, double>::value, double2, float2>::type T2;
      T2 t;
      t.x = static_cast<S>(v[0]); t.y = static_cast<S>(v[1]);
      *reinterpret_cast<T2*>(p) = t;
    }
  }
}

// Thread t of block b: rows are (o * n_out + i); a row has inner/4 vector
// slots.  When a row has fewer than TPB slots, a block packs TPB / slots
// rows; otherwise a row spans kchunks blocks.
template <class S, class C, int WC, int VEC>
__global__ void __launch_bounds__(TPB) k_gather_v4(const int* __restrict__ col, const C* __restrict__ coef, int Wr,
                                                   int n_out, const S* __restrict__ x, S* __restrict__ y,
                                                   uint32_t inner, int n_in, int in_base, C alpha, C beta,
                                                   uint32_t nrows, uint32_t slots, uint32_t rpb, uint32_t kchunks) {
  const int W = WC > 0 ? WC : Wr;
  uint32_t row, slot;
  if (rpb > 1) {
    row = blockIdx.x * rpb + threadIdx.x / slots;
    slot = threadIdx.x % slots;
    if (threadIdx.x >= rpb * slots) return;
  } else {
    row = blockIdx.x / kchunks;
    slot = (blockIdx.x % kchunks) * TPB + threadIdx.x;
    if (slot >= slots) return;
  }
  if (row >= nrows) return;
  const uint32_t k = slot * VEC;
  const int i = static_cast<int>(row % static_cast<uint32_t>(n_out));
  const uint32_t o = row / static_cast<uint32_t>(n_out);
  const int* cr = col + static_cast<int64_t>(i) * W;
  const C* cf = coef + static_cast<int64_t>(i) * W;
  const S* xb = x + (static_cast<int64_t>(o) * n_in) * inner + k;
  C acc[VEC];
#pragma unroll
  for (int e = 0; e < VEC; ++e) acc[e] = C(0);
  if (WC > 0) {
    // all loads of the row issued before the arithmetic
    C v[WC > 0 ? WC : 1][VEC];
    C a[WC > 0 ? WC : 1];
#pragma unroll
    for (int w = 0; w < WC; ++w) {
      const int c = cr[w] - in_base;
      const bool ok = static_cast<unsigned>(c) < static_cast<unsigned>(n_in);
      a[w] = ok ? cf[w] : C(0);
      loadv<VEC, S, C>(xb + static_cast<int64_t>(ok ? c : 0) * inner, v[w]);
    }
#pragma unroll
    for (int w = 0; w < WC; ++w)
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[e] += a[w] * v[w][e];
  } else {
    for (int w = 0; w < W; ++w) {
      const int c = cr[w] - in_base;
      if (static_cast<unsigned>(c) < static_cast<unsigned>(n_in)) {
        C v[VEC];
        loadv<VEC, S, C>(xb + static_cast<int64_t>(c) * inner, v);
        const C a = cf[w];
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] += a * v[e];
      }
    }
  }
  S* yp = y + static_cast<int64_t>(row) * inner + k;
  C r[VEC];
  if (beta != C(0)) {
    C old[VEC];
    loadv<VEC, S, C>(yp, old);
#pragma unroll
    for (int e = 0; e < VEC; ++e) r[e] = alpha * acc[e] + beta * old[e];
  } else {
#pragma unroll
    for (int e = 0; e < VEC; ++e) r[e] = alpha * acc[e];
  }
  storev<VEC, S, C>(yp, r);
}


// Column sweep for tables whose rows read contiguous, non-decreasing windows
// [c0[i], c0[i] + W): one thread owns VEC consecutive k of one outer index and
// a chunk of output rows, keeps the W input rows of the current window in
// registers and loads each new input row once as the window slides.  Every
// input row is fetched once per chunk (plus W-1 rows of overlap) and every
// output once, so the cache traffic equals the algorithmic traffic.
template <class S, class C, int W, int VEC>
__global__ void __launch_bounds__(TPB) k_sweep(const int* __restrict__ c0, const C* __restrict__ coef, int n_out,
                                               const S* __restrict__ x, S* __restrict__ y, uint32_t inner, int n_in,
                                               int in_base, C alpha, C beta, uint32_t slots, int rc, uint32_t nchunks,
                                               uint32_t total) {
  const uint32_t tid = blockIdx.x * TPB + threadIdx.x;
  if (tid >= total) return;
  const uint32_t slot = tid % slots;
  const uint32_t rest = tid / slots;
  const uint32_t chunk = rest % nchunks;
  const uint32_t o = rest / nchunks;
  const int i0 = static_cast<int>(chunk) * rc;
  const int i1 = min(n_out, i0 + rc);
  if (i0 >= i1) return;
  const uint32_t k = slot * VEC;
  const S* xb = x + static_cast<int64_t>(o) * n_in * inner + k;
  S* yb = y + static_cast<int64_t>(o) * n_out * inner + k;
  C ring[W][VEC];
  int base = c0[i0] - in_base;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const int r = base + w;
    if (static_cast<unsigned>(r) < static_cast<unsigned>(n_in)) loadv<VEC, S, C>(xb + static_cast<int64_t>(r) * inner, ring[w]);
    else
#pragma unroll
      for (int e = 0; e < VEC; ++e) ring[w][e] = C(0);
  }
  for (int i = i0; i < i1; ++i) {
    const int cb = c0[i] - in_base;
    while (base < cb) {
#pragma unroll
      for (int w = 0; w < W - 1; ++w)
#pragma unroll
        for (int e = 0; e < VEC; ++e) ring[w][e] = ring[w + 1][e];
      ++base;
      const int r = base + W - 1;
      if (static_cast<unsigned>(r) < static_cast<unsigned>(n_in)) loadv<VEC, S, C>(xb + static_cast<int64_t>(r) * inner, ring[W - 1]);
      else
#pragma unroll
        for (int e = 0; e < VEC; ++e) ring[W - 1][e] = C(0);
    }
    const C* cf = coef + static_cast<int64_t>(i) * W;
    C acc[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] = C(0);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const C a = cf[w];
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[e] += a * ring[w][e];
    }
    S* yp = yb + static_cast<int64_t>(i) * inner;
    C r[VEC];
    if (beta != C(0)) {
      C old[VEC];
      loadv<VEC, S, C>(yp, old);
#pragma unroll
      for (int e = 0; e < VEC; ++e) r[e] = alpha * acc[e] + beta * old[e];
    } else {
#pragma unroll
      for (int e = 0; e < VEC; ++e) r[e] = alpha * acc[e];
    }
    storev<VEC, S, C>(yp, r);
  }
}

// Column-sweep for any inner extent: the (outer, inner) columns are
// flattened and lane l of a wave owns columns base + l + 64 e (e < E), so
// every load and store instruction is coalesced whatever the alignment of
// inner; the window logic is that of k_sweep.
template <class S, class C, int W, int E>
__global__ void __launch_bounds__(TPB) k_sweep_flat(const int* __restrict__ c0, const C* __restrict__ coef, int n_out,
                                                    const S* __restrict__ x, S* __restrict__ y, int64_t inner,
                                                    int n_in, int in_base, C alpha, C beta, int64_t ncols, int rc,
                                                    int nchunks) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * TPB + threadIdx.x) >> 6;
  const int chunk = static_cast<int>(wave % nchunks);
  const int64_t grp = wave / nchunks;
  const int i0 = chunk * rc;
  const int i1 = min(n_out, i0 + rc);
  if (i0 >= i1) return;
  int64_t xo[E], yo[E];
  bool ok[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int64_t c = grp * (64 * E) + lane + 64 * e;
    ok[e] = c < ncols;
    const int64_t cc = ok[e] ? c : 0;
    const int64_t o = cc / inner, k = cc - o * inner;
    xo[e] = o * n_in * inner + k;
    yo[e] = o * static_cast<int64_t>(n_out) * inner + k;
  }
  C ring[W][E];
  int base = c0[i0] - in_base;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const int r = base + w;
    const bool rin = static_cast<unsigned>(r) < static_cast<unsigned>(n_in);
#pragma unroll
    for (int e = 0; e < E; ++e) ring[w][e] = (rin && ok[e]) ? to_c(x[xo[e] + static_cast<int64_t>(r) * inner], C(0)) : C(0);
  }
  for (int i = i0; i < i1; ++i) {
    const int cb = c0[i] - in_base;
    while (base < cb) {
#pragma unroll
      for (int w = 0; w < W - 1; ++w)
#pragma unroll
        for (int e = 0; e < E; ++e) ring[w][e] = ring[w + 1][e];
      ++base;
      const int r = base + W - 1;
      const bool rin = static_cast<unsigned>(r) < static_cast<unsigned>(n_in);
#pragma unroll
      for (int e = 0; e < E; ++e)
        ring[W - 1][e] = (rin && ok[e]) ? to_c(x[xo[e] + static_cast<int64_t>(r) * inner], C(0)) : C(0);
    }
    const C* cf = coef + static_cast<int64_t>(i) * W;
    C acc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = C(0);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const C a = cf[w];
#pragma unroll
      for (int e = 0; e < E; ++e) acc[e] += a * ring[w][e];
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (!ok[e]) continue;
      S* yp = y + yo[e] + static_cast<int64_t>(i) * inner;
      C r = alpha * acc[e];
      if (beta != C(0)) r += beta * to_c(*yp, C(0));
      *yp = from_c<S>(r);
    }
  }
}

// Two tables P, Q with the same windows applied along one axis in one pass
// (flattened columns as in k_sweep_flat):
//   out1 = P x (when out1 is given),  out2 = alpha Q x + beta P z.
// One sweep of the constant Kronecker part needs exactly this at every axis
// after the first (mass and stiffness share their band).
template <class S, class C, int W, int E>
__global__ void __launch_bounds__(TPB) k_sweep_dual(const int* __restrict__ c0, const C* __restrict__ P,
                                                    const C* __restrict__ Q, int n_out, const S* __restrict__ x,
                                                    const S* __restrict__ z, S* __restrict__ out1,
                                                    S* __restrict__ out2, int64_t inner, int n_in, int in_base,
                                                    C alpha, C beta, int64_t ncols, int rc, int nchunks) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * TPB + threadIdx.x) >> 6;
  const int chunk = static_cast<int>(wave % nchunks);
  const int64_t grp = wave / nchunks;
  const int i0 = chunk * rc;
  const int i1 = min(n_out, i0 + rc);
  if (i0 >= i1) return;
  int64_t xo[E], yo[E];
  bool ok[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int64_t c = grp * (64 * E) + lane + 64 * e;
    ok[e] = c < ncols;
    const int64_t cc = ok[e] ? c : 0;
    const int64_t o = cc / inner, k = cc - o * inner;
    xo[e] = o * n_in * inner + k;
    yo[e] = o * static_cast<int64_t>(n_out) * inner + k;
  }
  C rx[W][E], rz[W][E];
  int base = c0[i0] - in_base;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const int r = base + w;
    const bool rin = static_cast<unsigned>(r) < static_cast<unsigned>(n_in);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int64_t off = xo[e] + static_cast<int64_t>(r) * inner;
      rx[w][e] = (rin && ok[e]) ? to_c(x[off], C(0)) : C(0);
      rz[w][e] = (rin && ok[e]) ? to_c(z[off], C(0)) : C(0);
    }
  }
  for (int i = i0; i < i1; ++i) {
    const int cb = c0[i] - in_base;
    while (base < cb) {
#pragma unroll
      for (int w = 0; w < W - 1; ++w)
#pragma unroll
        for (int e = 0; e < E; ++e) {
          rx[w][e] = rx[w + 1][e];
          rz[w][e] = rz[w + 1][e];
        }
      ++base;
      const int r = base + W - 1;
      const bool rin = static_cast<unsigned>(r) < static_cast<unsigned>(n_in);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int64_t off = xo[e] + static_cast<int64_t>(r) * inner;
        rx[W - 1][e] = (rin && ok[e]) ? to_c(x[off], C(0)) : C(0);
        rz[W - 1][e] = (rin && ok[e]) ? to_c(z[off], C(0)) : C(0);
      }
    }
    const C* pf = P + static_cast<int64_t>(i) * W;
    const C* qf = Q + static_cast<int64_t>(i) * W;
    C px[E], qx[E], pz[E];
#pragma unroll
    for (int e = 0; e < E; ++e) px[e] = qx[e] = pz[e] = C(0);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const C pw = pf[w], qw = qf[w];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        px[e] += pw * rx[w][e];
        qx[e] += qw * rx[w][e];
        pz[e] += pw * rz[w][e];
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (!ok[e]) continue;
      const int64_t off = yo[e] + static_cast<int64_t>(i) * inner;
      if (out1) out1[off] = from_c<S>(px[e]);
      out2[off] = from_c<S>(alpha * qx[e] + beta * pz[e]);
    }
  }
}

// Fastest-axis variant (inner == 1): the table is staged in LDS once per
// block; the block then loops over groups of RB consecutive input rows (one
// contiguous span, staged with coalesced 16-byte loads when aligned),
// produces the RB output rows from LDS and writes them contiguously.
template <class S, class C, int WT>
__global__ void __launch_bounds__(TPB) k_gather_rows(const int* __restrict__ col, const C* __restrict__ coef, int W,
                                                     int n_out, const S* __restrict__ x, S* __restrict__ y, int n_in,
                                                     int in_base, C alpha, C beta, int64_t nrows, int RB) {
  extern __shared__ char smem_raw[];
  // table staged tap-major ([w][i]) so that lanes reading consecutive output
  // rows hit consecutive LDS words
  C* cs = reinterpret_cast<C*>(smem_raw);                       // W * n_out coefficients
  int* is = reinterpret_cast<int*>(cs + n_out * W);             // W * n_out local columns
  S* xs = reinterpret_cast<S*>(smem_raw + ((static_cast<size_t>(n_out) * W * (sizeof(C) + sizeof(int)) + 15) & ~static_cast<size_t>(15)));
  for (int t = threadIdx.x; t < n_out * W; t += TPB) {
    const int i = t / W, w = t - i * W;
    const int c = col[t] - in_base;
    const bool ok = static_cast<unsigned>(c) < static_cast<unsigned>(n_in);
    cs[w * n_out + i] = ok ? coef[t] : C(0);
    is[w * n_out + i] = ok ? c : 0;
  }
  constexpr int V = 16 / sizeof(S);
  typedef struct { S v[V]; } __attribute__((aligned(16))) Vec;
  const int dq = TPB / n_out, dr = TPB - dq * n_out;
  for (int64_t r0 = static_cast<int64_t>(blockIdx.x) * RB; r0 < nrows; r0 += static_cast<int64_t>(gridDim.x) * RB) {
    const int rb = static_cast<int>(min(static_cast<int64_t>(RB), nrows - r0));
    const S* xb = x + r0 * n_in;
    const int span = rb * n_in;
    const int nv = (reinterpret_cast<uintptr_t>(xb) % 16 == 0) ? span / V : 0;
    __syncthreads();   // the previous group's reads of xs are done
    {
      const Vec* src = reinterpret_cast<const Vec*>(xb);
      Vec* dst = reinterpret_cast<Vec*>(xs);
      for (int t = threadIdx.x; t < nv; t += TPB) dst[t] = src[t];
    }
    for (int t = nv * V + threadIdx.x; t < span; t += TPB) xs[t] = xb[t];
    __syncthreads();
    S* yb = y + r0 * n_out;
    // output (row r, entry i) of flat index t, stepped by TPB without divisions
    int r = threadIdx.x / n_out, i = threadIdx.x - (threadIdx.x / n_out) * n_out;
    for (; r < rb;) {
      const S* xr = xs + r * n_in;
      C acc = C(0);
      if constexpr (WT > 0) {
#pragma unroll
        for (int w = 0; w < WT; ++w) acc += cs[w * n_out + i] * to_c(xr[is[w * n_out + i]], C(0));
      } else {
        for (int w = 0; w < W; ++w) acc += cs[w * n_out + i] * to_c(xr[is[w * n_out + i]], C(0));
      }
      const int t = r * n_out + i;
      C v = alpha * acc;
      if (beta != C(0)) v += beta * to_c(yb[t], C(0));
      yb[t] = from_c<S>(v);
      r += dq;
      i += dr;
      if (i >= n_out) {
        i -= n_out;
        ++r;
      }
    }
  }
}

__global__ void __launch_bounds__(TPB) k_mode_max(const int* __restrict__ start, const int* __restrict__ cnt,
                                                  int n_out, const double* __restrict__ x, double* __restrict__ y,
                                                  int64_t inner, int n_in, int64_t total) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int64_t k = idx % inner;
  const int64_t t = idx / inner;
  const int i = static_cast<int>(t % n_out);
  const int64_t o = t / n_out;
  const double* xb = x + o * static_cast<int64_t>(n_in) * inner + k;
  double m = 0.0;
  const int s0 = start[i], c = cnt[i];
  for (int w = 0; w < c; ++w) m = fmax(m, xb[static_cast<int64_t>(s0 + w) * inner]);
  y[idx] = m;
}

// ---------------------------------------------------------------- time mixing
template <class S, class C, int P>
__global__ void __launch_bounds__(TPB) k_time_mix(const C* __restrict__ T, const S* __restrict__ Psi, int r0, int R,
                                                  int Nt, int t0, int t1, const S* __restrict__ Z, int n_in,
                                                  int in_base, S* __restrict__ out, int64_t Qs) {
  extern __shared__ char smem_raw[];
  C* ps = reinterpret_cast<C*>(smem_raw);
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= Qs) return;
  for (int r = 0; r < R; ++r) ps[r * blockDim.x + threadIdx.x] = to_c(Psi[static_cast<int64_t>(r0 + r) * Qs + q], C(0));
  constexpr int WB = 2 * P + 1;
  C win[WB];
#pragma unroll
  for (int w = 0; w < WB; ++w) {
    const int j = t0 + 1 - P + w - in_base;
    win[w] = (static_cast<unsigned>(j) < static_cast<unsigned>(n_in)) ? to_c(Z[static_cast<int64_t>(j) * Qs + q], C(0)) : C(0);
  }
  for (int t = t0; t < t1; ++t) {
    C acc = C(0);
    for (int r = 0; r < R; ++r) {
      const C* Tr = T + (static_cast<int64_t>(r0 + r) * Nt + t) * WB;
      C s = C(0);
#pragma unroll
      for (int w = 0; w < WB; ++w) s += Tr[w] * win[w];
      acc += ps[r * blockDim.x + threadIdx.x] * s;
    }
    out[static_cast<int64_t>(t - t0) * Qs + q] = from_c<S>(acc);
#pragma unroll
    for (int w = 0; w < WB - 1; ++w) win[w] = win[w + 1];
    const int j = t + 2 + P - in_base;
    win[WB - 1] = (static_cast<unsigned>(j) < static_cast<unsigned>(n_in)) ? to_c(Z[static_cast<int64_t>(j) * Qs + q], C(0)) : C(0);
  }
}


// ---------------------------------------------------------------- exact reaction term
// Reaction (and shock-capturing) terms with coefficients known at every
// space-time Gauss point (Cq[g][q] = omega_g omega_q C_r at time Gauss point g
// and spatial Gauss point q; Rq the same for the shock-capturing coefficient),
// over one slab of output time rows:
//   out[t][q] = beta out[t][q]
//     + sum_{e in supp b_i} sum_{g in e} Bv(g, i) Cq[g][q] sum_a B(g, f_e + a) Z[f_e + a][q]
//     + sum_{e in supp b_i} sum_{g in e} B'(g, i) Rq[g][q] sum_a B'(g, f_e + a) Z[f_e + a][q]
// with i = t0 + t + 1 the full index of unknown row t0 + t, Bv the test
// values (b_i, or b_i + tau b_i' with SUPG) and B' the time derivatives.
// Either term is skipped when its coefficient is null.  Z holds the spatially
// expanded input layers of full indices [lo_full, lo_full + nl) (layers
// outside read as zero: the initial layer of an unknown vector).  One thread
// per (row, spatial point): consecutive threads take consecutive q, so every
// Z, Cq, Rq and out access of a wave is one contiguous segment.
template <class S, class C, int KP>
__global__ void __launch_bounds__(TPB) k_react_point(const S* __restrict__ Z, int nl, int lo_full,
                                                     const C* __restrict__ Bt, const C* __restrict__ Bv,
                                                     const C* __restrict__ Bd, const int* __restrict__ tfirst,
                                                     const int* __restrict__ re0, const int* __restrict__ re1,
                                                     const C* __restrict__ Cq, const C* __restrict__ Rq, int64_t Qs,
                                                     int t0, int rows, S* __restrict__ out, C beta) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(rows) * Qs) return;
  const int t = static_cast<int>(idx / Qs);
  const int64_t q = idx - static_cast<int64_t>(t) * Qs;
  const int i = t0 + t + 1;
  C acc = C(0);
  for (int e = re0[i]; e < re1[i]; ++e) {
    const int fe = tfirst[e * KP];
    C zl[KP];
#pragma unroll
    for (int a = 0; a < KP; ++a) {
      const int j = fe + a - lo_full;
      zl[a] = (j >= 0 && j < nl) ? to_c(Z[static_cast<int64_t>(j) * Qs + q], C(0)) : C(0);
    }
    const int ai = i - fe;
#pragma unroll
    for (int g = 0; g < KP; ++g) {
      const int qg = e * KP + g;
      if (Cq) {
        C z = C(0);
#pragma unroll
        for (int a = 0; a < KP; ++a) z += Bt[qg * KP + a] * zl[a];
        acc += Bv[qg * KP + ai] * Cq[static_cast<int64_t>(qg) * Qs + q] * z;
      }
      if (Rq) {
        C z = C(0);
#pragma unroll
        for (int a = 0; a < KP; ++a) z += Bd[qg * KP + a] * zl[a];
        acc += Bd[qg * KP + ai] * Rq[static_cast<int64_t>(qg) * Qs + q] * z;
      }
    }
  }
  const int64_t o = static_cast<int64_t>(t) * Qs + q;
  out[o] = from_c<S>(beta != C(0) ? beta * to_c(out[o], C(0)) + acc : acc);
}

// ---------------------------------------------------------------- banded time solves
// Time direction of the preconditioner of the SUPG system: for every spatial
// mode j the banded N_t x N_t matrix T_j = A + (lam_j - shift) B (band
// half-width P, rows and columns of X_t; A and B stored as [t][2P + 1], column
// t - P + k) is factorized T_j = L_j U_j without pivoting (the symmetric part
// of T_j is positive definite: the time derivative with its initial condition,
// the SUPG time stiffness and non-negative reaction and diffusion terms), one
// thread per mode.  F[(t (2P + 1) + k) Ns + j]: k < P the multipliers
// l_{t, t-P+k}, k = P the reciprocal pivot, k > P the entries u_{t, t+k-P}.
template <int P>
__global__ void __launch_bounds__(TPB) k_band_factor(const double* __restrict__ A, const double* __restrict__ B,
                                                     int Nt, const double* __restrict__ lam, double shift, int64_t Ns,
                                                     double* __restrict__ F) {
  constexpr int KW = 2 * P + 1;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= Ns) return;
  const double lj = lam[j] - shift;
  double up[P][P + 1];   // U rows t - P .. t - 1 (diagonal first)
#pragma unroll
  for (int r = 0; r < P; ++r)
#pragma unroll
    for (int m = 0; m <= P; ++m) up[r][m] = 0.0;
  for (int t = 0; t < Nt; ++t) {
    double a[KW];
#pragma unroll
    for (int k = 0; k < KW; ++k) a[k] = A[t * KW + k] + lj * B[t * KW + k];
#pragma unroll
    for (int k = 0; k < P; ++k) {
      double l = 0.0;
      if (t - P + k >= 0) {
        l = a[k] / up[k][0];
#pragma unroll
        for (int m = 1; m <= P; ++m) a[k + m] -= l * up[k][m];
      }
      F[(static_cast<int64_t>(t) * KW + k) * Ns + j] = l;
    }
    F[(static_cast<int64_t>(t) * KW + P) * Ns + j] = 1.0 / a[P];
#pragma unroll
    for (int m = 1; m <= P; ++m) F[(static_cast<int64_t>(t) * KW + P + m) * Ns + j] = a[P + m];
#pragma unroll
    for (int r = 0; r < P - 1; ++r)
#pragma unroll
      for (int m = 0; m <= P; ++m) up[r][m] = up[r + 1][m];
#pragma unroll
    for (int m = 0; m <= P; ++m) up[P - 1][m] = a[P + m];
  }
}

// x_j = T_j^{-1} r_j with the factors of k_band_factor (layout [t][Ns] for r
// and x, which must not alias): forward substitution into x, then backward
// substitution in place, one thread per mode (each access of a wave is one
// contiguous segment).
template <class S, class C, int P>
__global__ void __launch_bounds__(TPB) k_band_solve(const C* __restrict__ F, int Nt, int64_t Ns,
                                                    const S* __restrict__ r, S* __restrict__ x) {
  constexpr int KW = 2 * P + 1;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= Ns) return;
  C ring[P];
#pragma unroll
  for (int k = 0; k < P; ++k) ring[k] = C(0);
  // unrolled: the loads of eight rows (independent of the recurrence) are in
  // flight together; with few spatial modes the walk is latency-bound
#pragma unroll 8
  for (int t = 0; t < Nt; ++t) {       // L y = r, ring = y_{t-P .. t-1}
    C y = to_c(r[static_cast<int64_t>(t) * Ns + j], C(0));
#pragma unroll
    for (int k = 0; k < P; ++k) y -= F[(static_cast<int64_t>(t) * KW + k) * Ns + j] * ring[k];
#pragma unroll
    for (int k = 0; k < P - 1; ++k) ring[k] = ring[k + 1];
    ring[P - 1] = y;
    x[static_cast<int64_t>(t) * Ns + j] = from_c<S>(y);
  }
#pragma unroll
  for (int k = 0; k < P; ++k) ring[k] = C(0);
#pragma unroll 8
  for (int t = Nt - 1; t >= 0; --t) {  // U x = y, ring = x_{t+1 .. t+P}
    C v = to_c(x[static_cast<int64_t>(t) * Ns + j], C(0));
#pragma unroll
    for (int m = 1; m <= P; ++m) v -= F[(static_cast<int64_t>(t) * KW + P + m) * Ns + j] * ring[m - 1];
    v *= F[(static_cast<int64_t>(t) * KW + P) * Ns + j];
#pragma unroll
    for (int m = P - 1; m > 0; --m) ring[m] = ring[m - 1];
    ring[0] = v;
    x[static_cast<int64_t>(t) * Ns + j] = from_c<S>(v);
  }
}

// ---------------------------------------------------------------- fused coefficient terms
// The low-rank coefficient terms along the slowest spatial axis in one pass:
// expansion of the input to the axis' Gauss points, the time mixing with the
// rank weights (as in k_time_mix) and the projection back onto the axis'
// B-splines, without storing Gauss-point arrays.  Z and out have layout
// [layer][nd][Qin] (Qin = Gauss points of the faster axes, already expanded).
// A thread owns one column c, TS consecutive output rows (blockIdx.y) and
// the B-spline range [d0, d1) of chunk blockIdx.z, whose elements are
// [e0, e1).  It walks the elements in order with a ring of the KP = p + 1
// input B-spline rows an element touches (each over the NL input layers the
// rows' time windows read) and a ring of their partial outputs; a B-spline is
// complete, and stored, once the walk has passed its last element.
// Block order of the fused coefficient kernels, XCD-aware: consecutive
// workgroups go to the 8 XCDs in turn, so the nslab time slabs of one column
// block (which read the same rank weights and overlapping input layers) are
// given ids 8 apart and run back to back on one XCD, sharing its L2.  The
// grid has ceil(ncb * nchunk / 8) * 8 * nslab blocks; the padding ones exit.
__device__ __forceinline__ bool coef_block(int nslab, int64_t ncb, int nchunk, int& slab, int64_t& cb, int& ch) {
  const int64_t L = blockIdx.x;
  const int64_t k = L >> 3;
  slab = static_cast<int>(k % nslab);
  const int64_t g = (k / nslab) * 8 + (L & 7);
  if (g >= ncb * nchunk) return false;
  cb = g % ncb;
  ch = static_cast<int>(g / ncb);
  return true;
}

// IX: element index type (uint32_t when every index of Z, out and Psi fits,
// which keeps the per-layer offsets in 32-bit registers; else int64_t).
template <class S, class C, int P, int KP, int TS, int RM, class IX>
__global__ void __launch_bounds__(256) k_coef_fused(const C* __restrict__ T, const S* __restrict__ Psi, int r0, int R,
                                                    int Nt, int t0, int t1, const S* __restrict__ Z, int n_in,
                                                    int in_base, const C* __restrict__ Bl,
                                                    const int* __restrict__ efirst, const int* __restrict__ chunks,
                                                    int nd, int64_t Qin, S* __restrict__ out, int64_t Qs, int nslab,
                                                    int64_t ncb, int nchunk) {
  int slab, ch;
  int64_t cb;
  if (!coef_block(nslab, ncb, nchunk, slab, cb, ch)) return;
  const int64_t c = cb * blockDim.x + threadIdx.x;
  if (c >= Qin) return;
  constexpr int WB = 2 * P + 1, NL = TS + 2 * P;
  const int ta = t0 + slab * TS;
  const int e0 = chunks[4 * ch], e1 = chunks[4 * ch + 1];
  const int d0 = chunks[4 * ch + 2], d1 = chunks[4 * ch + 3];
  const int nrow = min(TS, t1 - ta);
  const int64_t lay = static_cast<int64_t>(nd) * Qin;
  const IX layI = static_cast<IX>(lay), QinI = static_cast<IX>(Qin), QsI = static_cast<IX>(Qs);
  const S* Zc = Z + c;
  S* oc = out + c;
  const S* Pc = Psi + c;
  const int jb = ta + 1 - P - in_base;   // input layer of window slot 0
  C zr[KP][NL], yr[KP][TS];
  int f = efirst[e0];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int dof = f + k;
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const int j = jb + l;
      zr[k][l] = (static_cast<unsigned>(j) < static_cast<unsigned>(n_in) && dof < nd)
                     ? to_c(Zc[static_cast<IX>(j) * layI + static_cast<IX>(dof) * QinI], C(0))
                     : C(0);
    }
#pragma unroll
    for (int t = 0; t < TS; ++t) yr[k][t] = C(0);
  }
  for (int e = e0; e < e1; ++e) {
    const int fn = efirst[e];
    for (; f < fn; ++f) {
      if (f >= d0 && f < d1) {
        S* o = oc + (static_cast<IX>(ta - t0) * layI + static_cast<IX>(f) * QinI);
#pragma unroll
        for (int t = 0; t < TS; ++t)
          if (t < nrow) o[static_cast<IX>(t) * layI] = from_c<S>(yr[0][t]);
      }
#pragma unroll
      for (int k = 0; k < KP - 1; ++k) {
#pragma unroll
        for (int l = 0; l < NL; ++l) zr[k][l] = zr[k + 1][l];
#pragma unroll
        for (int t = 0; t < TS; ++t) yr[k][t] = yr[k + 1][t];
      }
      const int dof = f + KP;
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        const int j = jb + l;
        zr[KP - 1][l] = (static_cast<unsigned>(j) < static_cast<unsigned>(n_in) && dof < nd)
                            ? to_c(Zc[static_cast<IX>(j) * layI + static_cast<IX>(dof) * QinI], C(0))
                            : C(0);
      }
#pragma unroll
      for (int t = 0; t < TS; ++t) yr[KP - 1][t] = C(0);
    }
    // RM > 0 (R <= RM): the element's rank weights are loaded up front, so
    // their latency is paid once per element instead of once per rank
    C pv[KP][RM > 0 ? RM : 1];
    if constexpr (RM > 0) {
      const S* pe = Pc + (static_cast<IX>(r0) * QsI + static_cast<IX>(e * KP) * QinI);
#pragma unroll
      for (int g = 0; g < KP; ++g)
#pragma unroll
        for (int r = 0; r < RM; ++r)
          pv[g][r] = (r < R) ? to_c(pe[static_cast<IX>(r) * QsI + static_cast<IX>(g) * QinI], C(0)) : C(0);
    }
#pragma unroll
    for (int g = 0; g < KP; ++g) {
      const int qd = e * KP + g;
      C b[KP];
#pragma unroll
      for (int k = 0; k < KP; ++k) b[k] = Bl[qd * KP + k];
      C zg[NL];
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        C v = C(0);
#pragma unroll
        for (int k = 0; k < KP; ++k) v += b[k] * zr[k][l];
        zg[l] = v;
      }
      C m[TS];
#pragma unroll
      for (int t = 0; t < TS; ++t) m[t] = C(0);
      auto mix = [&](int r, C psi) {
        const C* Tr = T + (static_cast<int64_t>(r0 + r) * Nt + ta) * WB;
#pragma unroll
        for (int t = 0; t < TS; ++t) {
          const C* Tt = Tr + t * WB;
          C sacc = C(0);
#pragma unroll
          for (int w = 0; w < WB; ++w) sacc += Tt[w] * zg[t + w];
          m[t] += psi * sacc;
        }
      };
      if constexpr (RM > 0) {
#pragma unroll
        for (int r = 0; r < RM; ++r)
          if (r < R) mix(r, pv[g][r]);
      } else {
        const S* ps = Pc + (static_cast<IX>(r0) * QsI + static_cast<IX>(qd) * QinI);
        for (int r = 0; r < R; ++r) mix(r, to_c(ps[static_cast<IX>(r) * QsI], C(0)));
      }
#pragma unroll
      for (int k = 0; k < KP; ++k)
#pragma unroll
        for (int t = 0; t < TS; ++t) yr[k][t] += b[k] * m[t];
    }
  }
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int dof = f + k;
    if (dof >= d0 && dof < d1 && dof < nd) {
      S* o = oc + (static_cast<IX>(ta - t0) * layI + static_cast<IX>(dof) * QinI);
#pragma unroll
      for (int t = 0; t < TS; ++t)
        if (t < nrow) o[static_cast<IX>(t) * layI] = from_c<S>(yr[k][t]);
    }
  }
}


// Same computation with the next element's input row and rank weights
// loaded one element ahead (more registers, fewer exposed load latencies;
// used in FP64, where occupancy is low anyway).
template <class S, class C, int P, int KP, int TS, int RM, bool PF>
__global__ void __launch_bounds__(256) k_coef_fused_pf(const C* __restrict__ T, const S* __restrict__ Psi, int r0, int R,
                                                    int Nt, int t0, int t1, const S* __restrict__ Z, int n_in,
                                                    int in_base, const C* __restrict__ Bl,
                                                    const int* __restrict__ efirst, const int* __restrict__ chunks,
                                                    int nd, int64_t Qin, S* __restrict__ out, int64_t Qs, int nslab,
                                                    int64_t ncb, int nchunk) {
  int slab, ch;
  int64_t cb;
  if (!coef_block(nslab, ncb, nchunk, slab, cb, ch)) return;
  const int64_t c = cb * blockDim.x + threadIdx.x;
  if (c >= Qin) return;
  constexpr int WB = 2 * P + 1, NL = TS + 2 * P;
  const int ta = t0 + slab * TS;
  const int e0 = chunks[4 * ch], e1 = chunks[4 * ch + 1];
  const int d0 = chunks[4 * ch + 2], d1 = chunks[4 * ch + 3];
  const int nrow = min(TS, t1 - ta);
  const int64_t lay = static_cast<int64_t>(nd) * Qin;
  const int jb = ta + 1 - P - in_base;   // input layer of window slot 0
  // one B-spline row of the input over the NL window layers
  auto load_row = [&](C* row, int dof) {
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const int j = jb + l;
      row[l] = (static_cast<unsigned>(j) < static_cast<unsigned>(n_in) && dof < nd)
                   ? to_c(Z[j * lay + static_cast<int64_t>(dof) * Qin + c], C(0))
                   : C(0);
    }
  };
  // rank weights of the KP Gauss points of element e (RM > 0: all R <= RM of them)
  auto load_psi = [&](C (*pv)[RM > 0 ? RM : 1], int e) {
    if constexpr (RM > 0) {
      const S* ps = Psi + static_cast<int64_t>(r0) * Qs + static_cast<int64_t>(e) * KP * Qin + c;
#pragma unroll
      for (int g = 0; g < KP; ++g)
#pragma unroll
        for (int r = 0; r < RM; ++r)
          pv[g][r] = (r < R) ? to_c(ps[static_cast<int64_t>(r) * Qs + static_cast<int64_t>(g) * Qin], C(0)) : C(0);
    }
  };
  C zr[KP][NL], yr[KP][TS];
  int f = efirst[e0];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    load_row(zr[k], f + k);
#pragma unroll
    for (int t = 0; t < TS; ++t) yr[k][t] = C(0);
  }
  // PF: prefetch, one element ahead, of the row entering the ring when the
  // next element starts one B-spline later (the usual case) and of its rank
  // weights; this costs registers, so it pays where occupancy is low anyway
  C nx[PF ? NL : 1];
  int nxdof = -1;
  C pv[KP][RM > 0 ? RM : 1], pn[KP][RM > 0 && PF ? RM : 1];
  if constexpr (PF) load_psi(pv, e0);
  for (int e = e0; e < e1; ++e) {
    const int fn = efirst[e];
    if (PF && fn == f + 1 && nxdof == f + KP) {
      if (f >= d0 && f < d1) {
        S* o = out + static_cast<int64_t>(ta - t0) * lay + static_cast<int64_t>(f) * Qin + c;
#pragma unroll
        for (int t = 0; t < TS; ++t)
          if (t < nrow) o[t * lay] = from_c<S>(yr[0][t]);
      }
#pragma unroll
      for (int k = 0; k < KP - 1; ++k) {
#pragma unroll
        for (int l = 0; l < NL; ++l) zr[k][l] = zr[k + 1][l];
#pragma unroll
        for (int t = 0; t < TS; ++t) yr[k][t] = yr[k + 1][t];
      }
#pragma unroll
      for (int l = 0; l < NL; ++l) zr[KP - 1][l] = nx[l];
#pragma unroll
      for (int t = 0; t < TS; ++t) yr[KP - 1][t] = C(0);
      f = fn;
    }
    for (; f < fn; ++f) {
      if (f >= d0 && f < d1) {
        S* o = out + static_cast<int64_t>(ta - t0) * lay + static_cast<int64_t>(f) * Qin + c;
#pragma unroll
        for (int t = 0; t < TS; ++t)
          if (t < nrow) o[t * lay] = from_c<S>(yr[0][t]);
      }
#pragma unroll
      for (int k = 0; k < KP - 1; ++k) {
#pragma unroll
        for (int l = 0; l < NL; ++l) zr[k][l] = zr[k + 1][l];
#pragma unroll
        for (int t = 0; t < TS; ++t) yr[k][t] = yr[k + 1][t];
      }
      load_row(zr[KP - 1], f + KP);
#pragma unroll
      for (int t = 0; t < TS; ++t) yr[KP - 1][t] = C(0);
    }
    // issue the next element's loads before this element's arithmetic
    if constexpr (PF) {
      nxdof = -1;
      if (e + 1 < e1) {
        if (efirst[e + 1] == fn + 1) {
          nxdof = fn + KP;
          load_row(nx, nxdof);
        }
        load_psi(pn, e + 1);
      }
    }
#pragma unroll
    for (int g = 0; g < KP; ++g) {
      const int qd = e * KP + g;
      C b[KP];
#pragma unroll
      for (int k = 0; k < KP; ++k) b[k] = Bl[qd * KP + k];
      C zg[NL];
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        C v = C(0);
#pragma unroll
        for (int k = 0; k < KP; ++k) v += b[k] * zr[k][l];
        zg[l] = v;
      }
      C m[TS];
#pragma unroll
      for (int t = 0; t < TS; ++t) m[t] = C(0);
      auto mix = [&](int r, C psi) {
        const C* Tr = T + (static_cast<int64_t>(r0 + r) * Nt + ta) * WB;
#pragma unroll
        for (int t = 0; t < TS; ++t) {
          const C* Tt = Tr + t * WB;
          C sacc = C(0);
#pragma unroll
          for (int w = 0; w < WB; ++w) sacc += Tt[w] * zg[t + w];
          m[t] += psi * sacc;
        }
      };
      if constexpr (RM > 0 && PF) {
#pragma unroll
        for (int r = 0; r < RM; ++r)
          if (r < R) mix(r, pv[g][r]);
      } else {
        const S* ps = Psi + static_cast<int64_t>(r0) * Qs + static_cast<int64_t>(qd) * Qin + c;
        for (int r = 0; r < R; ++r) mix(r, to_c(ps[static_cast<int64_t>(r) * Qs], C(0)));
      }
#pragma unroll
      for (int k = 0; k < KP; ++k)
#pragma unroll
        for (int t = 0; t < TS; ++t) yr[k][t] += b[k] * m[t];
    }
    if constexpr (RM > 0 && PF) {
#pragma unroll
      for (int g = 0; g < KP; ++g)
#pragma unroll
        for (int r = 0; r < RM; ++r) pv[g][r] = pn[g][r];
    }
  }
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int dof = f + k;
    if (dof >= d0 && dof < d1 && dof < nd) {
      S* o = out + static_cast<int64_t>(ta - t0) * lay + static_cast<int64_t>(dof) * Qin + c;
#pragma unroll
      for (int t = 0; t < TS; ++t)
        if (t < nrow) o[t * lay] = from_c<S>(yr[k][t]);
    }
  }
}


// ---------------------------------------------------------------- dense mode product on MFMA
// Y[o][i][k] = sum_j A[i][j] X[o][j][k] as a GEMM D = A X_cols over the
// columns c = (o, k).  Each wave owns 16 columns and every output row (n
// padded to NT*16); the K loop steps over j by 4 with the 16x16x4 MFMA
// (FP64 or FP32 accumulate).  Operand layouts of v_mfma_*_16x16x4: A lane l
// holds A[l%16][l/16], B lane l holds B[l/16][l%16]; result element v of lane
// l is D[4*(l/16)+v][l%16] for the FP32 form and D[l/16+4v][l%16] for the
// FP64 form (checked on gfx950).  A is zero-padded to npad x npad; X rows j >= n and
// columns c >= ncols read as 0, so all loads stay in bounds.
typedef double dx4 __attribute__((ext_vector_type(4)));
typedef float fx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dx4 mfma16x16x4(double a, double b, dx4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ fx4 mfma16x16x4(float a, float b, fx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <class C> struct Acc4;
template <> struct Acc4<double> { typedef dx4 T; };
template <> struct Acc4<float> { typedef fx4 T; };

// Row stride of the matrix in LDS: npad plus 16 bytes.  A wave reads rows
// t*16 + l%16 at column j + l/16; with a stride of npad (a multiple of 16
// elements) the 16 rows fall into one bank (16-way conflict), with 16 bytes
// more every lane of an access hits its own bank, in FP32 and FP64.
template <class C>
__host__ __device__ constexpr int lds_stride(int npad) {
  return npad + static_cast<int>(16 / sizeof(C));
}
// Copy of the padded npad x npad matrix into LDS (row stride lds_stride)
// with 16-byte loads, several in flight per thread (npad is a multiple of
// 16, the source 16-byte aligned).
template <class C>
__device__ __forceinline__ void stage_matrix(const C* __restrict__ Ap, C* As, int npad) {
  constexpr int V = 16 / sizeof(C);
  typedef struct { C v[V]; } __attribute__((aligned(16))) Vec;
  const Vec* src = reinterpret_cast<const Vec*>(Ap);
  Vec* dst = reinterpret_cast<Vec*>(As);
  const int vpr = npad / V;          // 16-byte vectors per row
  const int nv = npad * vpr;
#pragma unroll 8
  for (int t = threadIdx.x; t < nv; t += blockDim.x) dst[t + t / vpr] = src[t];
  __syncthreads();
}

template <class S, class C, int NT, bool LDS_A>
__global__ void __launch_bounds__(256) k_dense_mode(const C* __restrict__ Ap, int n, int npad,
                                                    const S* __restrict__ x, S* __restrict__ y, int64_t inner,
                                                    int64_t ncols) {
  extern __shared__ char smem_raw[];
  C* As = reinterpret_cast<C*>(smem_raw);
  if (LDS_A) {
    stage_matrix<C>(Ap, As, npad);
  }
  const C* Asrc = LDS_A ? As : Ap;
  const int lda = LDS_A ? lds_stride<C>(npad) : npad;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t c = (static_cast<int64_t>(blockIdx.x) * 4 + wv) * 16 + (lane & 15);
  const bool cv = c < ncols;
  const int64_t o = cv ? c / inner : 0;
  const int64_t kq = cv ? c - o * inner : 0;
  const S* xb = x + o * static_cast<int64_t>(n) * inner + kq;
  typedef typename Acc4<C>::T A4;
  A4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = A4{0, 0, 0, 0};
  const int r16 = lane & 15, q4 = lane >> 4;
  for (int kk = 0; kk < ((n + 3) & ~3); kk += 4) {
    const int j = kk + q4;
    const C b = (cv && j < n) ? to_c(xb[static_cast<int64_t>(j) * inner], C(0)) : C(0);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const C a = Asrc[(t * 16 + r16) * lda + j];
      acc[t] = mfma16x16x4(a, b, acc[t]);
    }
  }
  if (!cv) return;
  S* yb = y + o * static_cast<int64_t>(n) * inner + kq;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = t * 16 + (std::is_same<C, double>::value ? q4 + 4 * v : 4 * q4 + v);
      if (i < n) yb[static_cast<int64_t>(i) * inner] = from_c<S>(acc[t][v]);
    }
}


// Variant for inner % E == 0 (E = 2 or 4): a wave owns 16E columns as E
// 16-column MFMA tiles; lane l feeds columns c0 + E(l%16) + e of tile e from
// one E-wide load and stores the E results of a row with one E-wide store.
template <class S, class C, int NT, int E, bool LDS_A>
__global__ void __launch_bounds__(256) k_dense_modeE(const C* __restrict__ Ap, int n, int npad,
                                                     const S* __restrict__ x, S* __restrict__ y, int64_t inner,
                                                     int64_t ncols) {
  extern __shared__ char smem_raw[];
  C* As = reinterpret_cast<C*>(smem_raw);
  if (LDS_A) stage_matrix<C>(Ap, As, npad);
  const C* Asrc = LDS_A ? As : Ap;
  const int lda = LDS_A ? lds_stride<C>(npad) : npad;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r16 = lane & 15, q4 = lane >> 4;
  // persistent: the block walks groups of 4 waves' columns, staging A once
  const int64_t ngroups = (ncols + 64 * E - 1) / (64 * E);
  auto body = [&](int64_t grp) {
    const int64_t c = (grp * 4 + wv) * (16 * E) + E * r16;
    const bool cv = c < ncols;
    const int64_t o = cv ? c / inner : 0;
    const int64_t kq = cv ? c - o * inner : 0;
    const S* xb = x + o * static_cast<int64_t>(n) * inner + kq;
    typedef typename Acc4<C>::T A4;
    A4 acc[NT][E];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int e = 0; e < E; ++e) acc[t][e] = A4{0, 0, 0, 0};
    for (int kk = 0; kk < ((n + 3) & ~3); kk += 4) {
      const int j = kk + q4;
      C b[E];
      const bool ok = cv && j < n;
      loadv<E, S, C>(xb + static_cast<int64_t>(ok ? j : 0) * inner, b);
#pragma unroll
      for (int e = 0; e < E; ++e) b[e] = ok ? b[e] : C(0);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const C av = Asrc[(t * 16 + r16) * lda + j];
#pragma unroll
        for (int e = 0; e < E; ++e) acc[t][e] = mfma16x16x4(av, b[e], acc[t][e]);
      }
    }
    if (cv) {
      S* yb = y + o * static_cast<int64_t>(n) * inner + kq;
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = t * 16 + (std::is_same<C, double>::value ? q4 + 4 * v : 4 * q4 + v);
          if (i < n) {
            C r[E];
#pragma unroll
            for (int e = 0; e < E; ++e) r[e] = acc[t][e][v];
            storev<E, S, C>(yb + static_cast<int64_t>(i) * inner, r);
          }
        }
    }
  };
  // with the matrix in LDS the block walks several groups (staging it once);
  // otherwise each block owns exactly one group
  if constexpr (LDS_A) {
    for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) body(grp);
  } else {
    body(blockIdx.x);
  }
}

// Variant for any inner extent: the (outer, inner) columns are flattened; a
// wave owns 16E consecutive columns as E MFMA tiles, lane l feeding column
// base + 16 e + l%16 of tile e, so each load instruction reads 16
// consecutive columns of 4 rows whatever the alignment of inner.
template <class S, class C, int NT, int E, bool LDS_A>
__global__ void __launch_bounds__(256) k_dense_modeU(const C* __restrict__ Ap, int n, int npad,
                                                     const S* __restrict__ x, S* __restrict__ y, int64_t inner,
                                                     int64_t ncols) {
  extern __shared__ char smem_raw[];
  C* As = reinterpret_cast<C*>(smem_raw);
  if (LDS_A) stage_matrix<C>(Ap, As, npad);
  const C* Asrc = LDS_A ? As : Ap;
  const int lda = LDS_A ? lds_stride<C>(npad) : npad;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r16 = lane & 15, q4 = lane >> 4;
  const int n4 = (n + 3) & ~3;
  // persistent: the block walks groups of 4 waves' columns, staging A once
  const int64_t ngroups = (ncols + 64 * E - 1) / (64 * E);
  auto body = [&](int64_t grp) {
    const int64_t base = (grp * 4 + wv) * (16 * E) + r16;
    int64_t off[E];
    bool ok[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int64_t c = base + 16 * e;
      ok[e] = c < ncols;
      const int64_t cc = ok[e] ? c : 0;
      const int64_t o = cc / inner;
      off[e] = o * static_cast<int64_t>(n) * inner + (cc - o * inner);
    }
    typedef typename Acc4<C>::T A4;
    A4 acc[NT][E];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int e = 0; e < E; ++e) acc[t][e] = A4{0, 0, 0, 0};
    for (int kk = 0; kk < n4; kk += 4) {
      const int j = kk + q4;
      C b[E];
#pragma unroll
      for (int e = 0; e < E; ++e)
        b[e] = (j < n && ok[e]) ? to_c(x[off[e] + static_cast<int64_t>(j) * inner], C(0)) : C(0);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const C av = Asrc[(t * 16 + r16) * lda + j];
#pragma unroll
        for (int e = 0; e < E; ++e) acc[t][e] = mfma16x16x4(av, b[e], acc[t][e]);
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = t * 16 + (std::is_same<C, double>::value ? q4 + 4 * v : 4 * q4 + v);
        if (i < n) {
#pragma unroll
          for (int e = 0; e < E; ++e)
            if (ok[e]) y[off[e] + static_cast<int64_t>(i) * inner] = from_c<S>(acc[t][e][v]);
        }
      }
  };
  // with the matrix in LDS the block walks several groups (staging it once);
  // otherwise each block owns exactly one group
  if constexpr (LDS_A) {
    for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) body(grp);
  } else {
    body(blockIdx.x);
  }
}

// Variant for inner == 1 (the fastest axis): a one-wave block stages 16E
// consecutive rows x[o][0..n) (one contiguous span) in LDS with coalesced
// loads, multiplies them as E MFMA column tiles (each A fragment serves E
// products), writes the results back over the staged rows and stores the
// span coalesced.
template <class S, class C, int NT, int E>
__global__ void __launch_bounds__(64) k_dense_rows(const C* __restrict__ Ap, int n, int npad, const S* __restrict__ x,
                                                   S* __restrict__ y, int64_t outer) {
  extern __shared__ char smem_raw[];
  S* Xs = reinterpret_cast<S*>(smem_raw);
  constexpr int RB = 16 * E;
  const int64_t o0 = static_cast<int64_t>(blockIdx.x) * RB;
  const int rows = static_cast<int>(min<int64_t>(RB, outer - o0));
  const int span = rows * n;
  const S* xs = x + o0 * n;
  // the span starts at a multiple of 16 n elements: 16-byte aligned when x is
  constexpr int V = 16 / sizeof(S);
  typedef struct { S v[V]; } __attribute__((aligned(16))) Vec;
  const int lane = threadIdx.x;
  const int nv = (reinterpret_cast<uintptr_t>(xs) % 16 == 0) ? span / V : 0;
  {
    const Vec* src = reinterpret_cast<const Vec*>(xs);
    Vec* dst = reinterpret_cast<Vec*>(Xs);
#pragma unroll 4
    for (int t = lane; t < nv; t += 64) dst[t] = src[t];
  }
  for (int t = nv * V + lane; t < span; t += 64) Xs[t] = xs[t];
  __syncthreads();
  const int r16 = lane & 15, q4 = lane >> 4;
  typedef typename Acc4<C>::T A4;
  A4 acc[NT][E];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int e = 0; e < E; ++e) acc[t][e] = A4{0, 0, 0, 0};
  const int n4 = (n + 3) & ~3;
  for (int kk = 0; kk < n4; kk += 4) {
    const int j = kk + q4;
    C b[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int rr = 16 * e + r16;
      b[e] = (rr < rows && j < n) ? to_c(Xs[rr * n + j], C(0)) : C(0);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const C av = Ap[(t * 16 + r16) * npad + j];
#pragma unroll
      for (int e = 0; e < E; ++e) acc[t][e] = mfma16x16x4(av, b[e], acc[t][e]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int rr = 16 * e + r16;
    if (rr < rows) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = t * 16 + (std::is_same<C, double>::value ? q4 + 4 * v : 4 * q4 + v);
          if (i < n) Xs[rr * n + i] = from_c<S>(acc[t][e][v]);
        }
    }
  }
  __syncthreads();
  S* ys = y + o0 * n;
  const int mv = (reinterpret_cast<uintptr_t>(ys) % 16 == 0) ? span / V : 0;
  {
    const Vec* src = reinterpret_cast<const Vec*>(Xs);
    Vec* dst = reinterpret_cast<Vec*>(ys);
#pragma unroll 4
    for (int t = lane; t < mv; t += 64) dst[t] = src[t];
  }
  for (int t = mv * V + lane; t < span; t += 64) ys[t] = Xs[t];
}

// ---------------------------------------------------------------- dense mode product, BF16 on MFMA
// The same mode products with BF16 operands and FP32 accumulation on
// v_mfma_f32_16x16x16bf16_1k (K = 16 per instruction): A lane l holds
// A[l%16][4(l/16) + 0..3], B lane l holds B[4(l/16) + 0..3][l%16], the result
// layout is that of the FP32 16x16x4 form (lane l: rows 4(l/16) + v of
// column l%16).  The matrix is the zero-padded BF16 copy, staged in LDS with
// rows padded by 16 bytes; rows j >= n of X read as 0.
typedef short bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ fx4 mfma16x16x16bf16(bf16x4 a, bf16x4 b, fx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__host__ __device__ constexpr int lds_stride_b16(int npad) { return npad + 8; }

__device__ __forceinline__ void stage_matrix_b16(const bf16* __restrict__ Ap, unsigned short* As, int npad) {
  typedef struct { unsigned short v[8]; } __attribute__((aligned(16))) Vec;
  const Vec* src = reinterpret_cast<const Vec*>(Ap);
  Vec* dst = reinterpret_cast<Vec*>(As);
  const int vpr = npad / 8;          // 16-byte vectors per row (row stride npad + 8 = (vpr + 1) vectors)
  const int nv = npad * vpr;
#pragma unroll 8
  for (int t = threadIdx.x; t < nv; t += blockDim.x) dst[t + t / vpr] = src[t];
  __syncthreads();
}

__device__ __forceinline__ unsigned short bf16_bits(bf16 v) { return __builtin_bit_cast(unsigned short, v); }
__device__ __forceinline__ bf16 bf16_from_bits(unsigned short v) { return __builtin_bit_cast(bf16, v); }

// inner % E == 0: a wave owns 16E columns as E tiles, lane l the E adjacent
// columns c0 + E(l%16) + e (one E x 2-byte load per row)
template <int NT, int E>
__global__ void __launch_bounds__(256) k_dense_modeE_b16(const bf16* __restrict__ Ap, int n, int npad,
                                                         const bf16* __restrict__ x, bf16* __restrict__ y,
                                                         int64_t inner, int64_t ncols) {
  extern __shared__ char smem_raw[];
  unsigned short* As = reinterpret_cast<unsigned short*>(smem_raw);
  stage_matrix_b16(Ap, As, npad);
  const int lda = lds_stride_b16(npad);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r16 = lane & 15, q4 = lane >> 4;
  const int64_t ngroups = (ncols + 64 * E - 1) / (64 * E);
  typedef struct { unsigned short v[E]; } __attribute__((aligned(2 * E))) Row;
  for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const int64_t c = (grp * 4 + wv) * (16 * E) + E * r16;
    const bool cv = c < ncols;
    const int64_t o = cv ? c / inner : 0;
    const int64_t kq = cv ? c - o * inner : 0;
    const bf16* xb = x + o * static_cast<int64_t>(n) * inner + kq;
    fx4 acc[NT][E];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int e = 0; e < E; ++e) acc[t][e] = fx4{0, 0, 0, 0};
    for (int kk = 0; kk < npad; kk += 16) {
      Row rv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int j = kk + 4 * q4 + i;
        if (cv && j < n) {
          rv[i] = *reinterpret_cast<const Row*>(xb + static_cast<int64_t>(j) * inner);
        } else {
#pragma unroll
          for (int e = 0; e < E; ++e) rv[i].v[e] = 0;
        }
      }
      bf16x4 bop[E];
#pragma unroll
      for (int e = 0; e < E; ++e)
        bop[e] = bf16x4{static_cast<short>(rv[0].v[e]), static_cast<short>(rv[1].v[e]),
                        static_cast<short>(rv[2].v[e]), static_cast<short>(rv[3].v[e])};
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const bf16x4 aop = *reinterpret_cast<const bf16x4*>(As + (t * 16 + r16) * lda + kk + 4 * q4);
#pragma unroll
        for (int e = 0; e < E; ++e) acc[t][e] = mfma16x16x16bf16(aop, bop[e], acc[t][e]);
      }
    }
    if (cv) {
      bf16* yb = y + o * static_cast<int64_t>(n) * inner + kq;
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = t * 16 + 4 * q4 + v;
          if (i < n) {
            Row r;
#pragma unroll
            for (int e = 0; e < E; ++e) r.v[e] = bf16_bits(__float2bfloat16(acc[t][e][v]));
            *reinterpret_cast<Row*>(yb + static_cast<int64_t>(i) * inner) = r;
          }
        }
    }
  }
}

// inner == 1 (the fastest axis): a one-wave block stages 16E consecutive rows
// x[o][0..n) in LDS, multiplies them as E column tiles and writes the results
// back over the staged rows before the coalesced store
template <int NT, int E>
__global__ void __launch_bounds__(64) k_dense_rows_b16(const bf16* __restrict__ Ap, int n, int npad,
                                                       const bf16* __restrict__ x, bf16* __restrict__ y,
                                                       int64_t outer) {
  extern __shared__ char smem_raw[];
  unsigned short* Xs = reinterpret_cast<unsigned short*>(smem_raw);
  constexpr int RB = 16 * E;
  const int64_t o0 = static_cast<int64_t>(blockIdx.x) * RB;
  const int rows = static_cast<int>(min<int64_t>(RB, outer - o0));
  const int span = rows * n;
  const unsigned short* xs = reinterpret_cast<const unsigned short*>(x + o0 * n);
  const int lane = threadIdx.x;
  for (int t = lane; t < span; t += 64) Xs[t] = xs[t];
  __syncthreads();
  const int r16 = lane & 15, q4 = lane >> 4;
  fx4 acc[NT][E];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int e = 0; e < E; ++e) acc[t][e] = fx4{0, 0, 0, 0};
  const unsigned short* Au = reinterpret_cast<const unsigned short*>(Ap);
  for (int kk = 0; kk < npad; kk += 16) {
    bf16x4 bop[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int rr = 16 * e + r16;
      short v4[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int j = kk + 4 * q4 + i;
        v4[i] = (rr < rows && j < n) ? static_cast<short>(Xs[rr * n + j]) : static_cast<short>(0);
      }
      bop[e] = bf16x4{v4[0], v4[1], v4[2], v4[3]};
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const unsigned short* ar = Au + static_cast<int64_t>(t * 16 + r16) * npad + kk + 4 * q4;
      const bf16x4 aop = *reinterpret_cast<const bf16x4*>(ar);
#pragma unroll
      for (int e = 0; e < E; ++e) acc[t][e] = mfma16x16x16bf16(aop, bop[e], acc[t][e]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int rr = 16 * e + r16;
    if (rr < rows) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = t * 16 + 4 * q4 + v;
          if (i < n) Xs[rr * n + i] = bf16_bits(__float2bfloat16(acc[t][e][v]));
        }
    }
  }
  __syncthreads();
  unsigned short* ys = reinterpret_cast<unsigned short*>(y + o0 * n);
  for (int t = lane; t < span; t += 64) ys[t] = Xs[t];
}

// ---------------------------------------------------------------- arrowhead
template <class S, class C>
__global__ void __launch_bounds__(TPB) k_arrowhead(const S* __restrict__ r, S* __restrict__ y, const C* __restrict__ lam,
                                                   const C* __restrict__ mu, const C* __restrict__ l, C sigma, C Cm,
                                                   int Nt, int np, int64_t Ns) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= Ns) return;
  const C s = lam[j];
  const int n = Nt - 1;
  C acc = C(0), den = Cm * sigma + s;
  // the np 2x2 blocks come first, then 1x1 (zero-mode) blocks; the block
  // loops are unrolled so that several rows' loads are in flight together
#pragma unroll 4
  for (int q = 0; q < np; ++q) {
    const int a = 2 * q;
    const C dl = Cm * mu[a];
    const C inv = C(1) / (s * s + dl * dl);
    const C ra = to_c(r[static_cast<int64_t>(a) * Ns + j], C(0));
    const C rb = to_c(r[static_cast<int64_t>(a + 1) * Ns + j], C(0));
    const C la = l[a], lb = l[a + 1];
    acc += inv * (la * (s * ra - dl * rb) + lb * (dl * ra + s * rb));
    den += Cm * Cm * s * (la * la + lb * lb) * inv;
  }
  for (int a = 2 * np; a < n; ++a) {
    const C ra = to_c(r[static_cast<int64_t>(a) * Ns + j], C(0));
    acc += l[a] * ra / s;
    den += Cm * Cm * l[a] * l[a] / s;
  }
  const C yN = (to_c(r[static_cast<int64_t>(n) * Ns + j], C(0)) + Cm * acc) / den;
  y[static_cast<int64_t>(n) * Ns + j] = from_c<S>(yN);
#pragma unroll 4
  for (int q = 0; q < np; ++q) {
    const int a = 2 * q;
    const C dl = Cm * mu[a];
    const C inv = C(1) / (s * s + dl * dl);
    const C ta = to_c(r[static_cast<int64_t>(a) * Ns + j], C(0)) - Cm * l[a] * yN;
    const C tb = to_c(r[static_cast<int64_t>(a + 1) * Ns + j], C(0)) - Cm * l[a + 1] * yN;
    y[static_cast<int64_t>(a) * Ns + j] = from_c<S>(inv * (s * ta - dl * tb));
    y[static_cast<int64_t>(a + 1) * Ns + j] = from_c<S>(inv * (dl * ta + s * tb));
  }
  for (int a = 2 * np; a < n; ++a)
    y[static_cast<int64_t>(a) * Ns + j] = from_c<S>((to_c(r[static_cast<int64_t>(a) * Ns + j], C(0)) - Cm * l[a] * yN) / s);
}

// ---------------------------------------------------------------- time core
// The time part of the FD preconditioner in one pass, FP32 arithmetic:
// for every spatial mode j, b = U_t^T x[., j] (MFMA over the Nt time rows),
// the arrowhead solve of k_arrowhead on b, and z[., j] = U_t y.  A block
// stages both padded time matrices in LDS once (row stride lds_stride);
// then every wave independently walks tiles of 16 consecutive spatial modes
// (persistent, no block barriers).  The first product takes its operand
// straight from registers (lane l loads rows 4 e + l/16 of column l%16: the
// MFMA B layout of K step e), prefetched one tile ahead; its result goes to
// the wave's LDS tile (row stride TC_W: at most 2-way bank conflicts for the
// result writes, the arrowhead's row reads and the second product's operand
// reads), where 4 lanes per column solve the arrowhead (lane & 3 takes every
// 4th block of the sums, combined by lane shuffles); the second product is
// stored from the accumulators.  Requires npad = 16 NT <= 64.
constexpr int TC_W = 18, TC_WAVES = 8;
// LDS accesses of one wave are performed in issue order; this only keeps the
// compiler from moving LDS accesses across the point
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
template <class S, int NT>
__global__ void __launch_bounds__(64 * TC_WAVES) k_time_core(const float* __restrict__ UtT, const float* __restrict__ Ut,
                                                           int Nt, int npad, const S* __restrict__ x,
                                                           S* __restrict__ z, int64_t Ns,
                                                           const float* __restrict__ lam, const float* __restrict__ mu,
                                                           int np, const float* __restrict__ l, float sigma, float Cm) {
  extern __shared__ char smem_raw[];
  const int lda = lds_stride<float>(npad);
  float* A1 = reinterpret_cast<float*>(smem_raw);
  float* A2 = A1 + npad * lda;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float* Tw = A2 + npad * lda + wv * npad * TC_W;
  stage_matrix<float>(UtT, A1, npad);
  stage_matrix<float>(Ut, A2, npad);
  const int r16 = lane & 15, q4 = lane >> 4;
  const int n4 = (Nt + 3) & ~3;
  const int64_t ntiles = (Ns + 15) / 16;
  const int64_t GW = static_cast<int64_t>(gridDim.x) * TC_WAVES;
  constexpr int PE = 4 * NT;   // K steps of 4 rows (Nt <= npad = 16 NT)
  float pre[PE];
  auto fetch = [&](int64_t tile) {
    const int64_t j = tile * 16 + r16;
#pragma unroll
    for (int e = 0; e < PE; ++e) {
      const int t = 4 * e + q4;
      pre[e] = (t < Nt && j < Ns) ? to_c(x[static_cast<int64_t>(t) * Ns + j], 0.f) : 0.f;
    }
  };
  typedef typename Acc4<float>::T A4;
  int64_t tile = static_cast<int64_t>(blockIdx.x) * TC_WAVES + wv;
  if (tile < ntiles) fetch(tile);
  for (; tile < ntiles; tile += GW) {
    const int64_t j0 = tile * 16;
    float b0[PE];
#pragma unroll
    for (int e = 0; e < PE; ++e) b0[e] = pre[e];
    if (tile + GW < ntiles) fetch(tile + GW);
    A4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = A4{0, 0, 0, 0};
    // b = U_t^T x (rows >= Nt of U_t^T are zero)
#pragma unroll
    for (int e = 0; e < PE; ++e) {
      if (4 * e >= Nt) break;
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = mfma16x16x4(A1[(t * 16 + r16) * lda + 4 * e + q4], b0[e], acc[t]);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) Tw[(t * 16 + 4 * q4 + v) * TC_W + r16] = acc[t][v];
    wave_lds_sync();
    {
      const int cc = lane >> 2, part = lane & 3;
      const int64_t j = j0 + cc;
      const float s = j < Ns ? lam[j] : 1.f;
      const int nA = Nt - 1;
      float sa = 0.f, sd = 0.f;
      for (int q = part; q < np; q += 4) {
        const int a = 2 * q;
        const float dl = Cm * mu[a];
        const float inv = 1.f / (s * s + dl * dl);
        const float ra = Tw[a * TC_W + cc], rb = Tw[(a + 1) * TC_W + cc];
        const float la = l[a], lb = l[a + 1];
        sa += inv * (la * (s * ra - dl * rb) + lb * (dl * ra + s * rb));
        sd += Cm * Cm * s * (la * la + lb * lb) * inv;
      }
      for (int a = 2 * np + part; a < nA; a += 4) {
        const float ra = Tw[a * TC_W + cc];
        sa += l[a] * ra / s;
        sd += Cm * Cm * l[a] * l[a] / s;
      }
      sa += __shfl_xor(sa, 1, 64);
      sa += __shfl_xor(sa, 2, 64);
      sd += __shfl_xor(sd, 1, 64);
      sd += __shfl_xor(sd, 2, 64);
      // the 4 lanes of a column read r_N (one instruction) before any writes y_N
      const float yN = (Tw[nA * TC_W + cc] + Cm * sa) / (Cm * sigma + s + sd);
      for (int q = part; q < np; q += 4) {
        const int a = 2 * q;
        const float dl = Cm * mu[a];
        const float inv = 1.f / (s * s + dl * dl);
        const float ta = Tw[a * TC_W + cc] - Cm * l[a] * yN;
        const float tb = Tw[(a + 1) * TC_W + cc] - Cm * l[a + 1] * yN;
        Tw[a * TC_W + cc] = inv * (s * ta - dl * tb);
        Tw[(a + 1) * TC_W + cc] = inv * (dl * ta + s * tb);
      }
      for (int a = 2 * np + part; a < nA; a += 4) Tw[a * TC_W + cc] = (Tw[a * TC_W + cc] - Cm * l[a] * yN) / s;
      if (part == 0) Tw[nA * TC_W + cc] = yN;
    }
    wave_lds_sync();
    // z = U_t y (rows >= Nt of the tile hold zeros of the first product)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = A4{0, 0, 0, 0};
    for (int kk = 0; kk < n4; kk += 4) {
      const float b = Tw[(kk + q4) * TC_W + r16];
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = mfma16x16x4(A2[(t * 16 + r16) * lda + kk + q4], b, acc[t]);
    }
    wave_lds_sync();   // the tile's reads are issued before the next tile's writes
    const int64_t j = j0 + r16;
    if (j < Ns) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = t * 16 + 4 * q4 + v;
          if (row < Nt) z[static_cast<int64_t>(row) * Ns + j] = from_c<S>(acc[t][v]);
        }
    }
  }
}

// ---------------------------------------------------------------- reductions
constexpr int RED_E = 16;                 // elements per thread
constexpr int64_t RED_CHUNK = static_cast<int64_t>(TPB) * RED_E;

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  return v;
}
// block-wide sum; result valid in thread 0
__device__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (blockDim.x >> 6); ++i) r += sh[i];
  return r;
}
__device__ double block_max(double v, double* sh) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (blockDim.x >> 6); ++i) r = fmax(r, sh[i]);
  return r;
}

// ---------------------------------------------------------------- FGMRES Givens rotations
// The small serial part of an Arnoldi step, fused with the reduction that
// finishes |w'|^2 (one block): the Hessenberg column updates of the delayed
// Gram-Schmidt scheme and the Givens rotations that turn the Hessenberg
// matrix into R and the start residual into g, so that |g[k+1]| is the
// residual estimate after k + 1 steps.  The block stages the rotations, the
// step's dots and the stored raw column j - 1 in LDS; one lane then runs the
// rotation chain (the running entry of the column in a register) and writes
// back.  Plain FP64 arithmetic without contraction into fused multiply-adds.
__global__ void __launch_bounds__(TPB) k_norm_givens(const double* __restrict__ part, int nb, double* __restrict__ D,
                                                     double* __restrict__ G, GivensLayout L, int m, int j) {
#pragma clang fp contract(off)
  __shared__ double sh[TPB / 64];
  __shared__ double lcs[64], lsn[64], dd[128], colA[66], colB[66], misc[2];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += TPB) acc += part[b];
  const double w2 = block_sum(acc, sh);   // as k_finalize_sum with k = 1
  const int t = threadIdx.x;
  if (t < m) {
    lcs[t] = G[L.cs + t];
    lsn[t] = G[L.sn + t];
  }
  if (t < 2 * j + 1) dd[t] = D[t];
  if (t < j) colA[t] = G[L.Hr + t * m + j - 1];
  if (t == 0) {
    misc[0] = G[L.gpre + (j > 0 ? j - 1 : 0)];
    misc[1] = G[L.ap];
  }
  __syncthreads();
  if (t != 0) return;
  D[256] = w2;
  double* out = G + L.out + (j & 1) * 8;
  const double alpha = D[128], h = D[129];
  // the stored next vector is the projected w divided by alpha
  const double beta = alpha * sqrt(fmax(w2, 0.0));
  out[0] = alpha;
  out[1] = h;
  out[2] = beta;
  out[3] = 0.0;
  out[4] = 0.0;
  out[5] = 0.0;
  if (!isfinite(alpha) || !isfinite(h) || !isfinite(beta)) {
    out[5] = 1.0;
    return;
  }
  // Givens rotation of column k (raw entries col[0..k+1]) by the rotations of
  // the columns before it and its own new rotation; returns g[k] and sets
  // g[k+1] (gnext) from the provisional entry gp = g[k] before rotation
  auto rotate = [&](double* col, int k, double gp, double& gk, double& gnext) {
    double carry = col[0];
    for (int i = 0; i < k; ++i) {
      const double t1 = carry, t2 = col[i + 1];
      col[i] = lcs[i] * t1 + lsn[i] * t2;
      carry = -lsn[i] * t1 + lcs[i] * t2;
    }
    const double hkk = carry, hn = col[k + 1];
    const double den = hypot(hkk, hn);
    const double c = den == 0.0 ? 1.0 : hkk / den;
    const double sv = den == 0.0 ? 0.0 : hn / den;
    col[k] = den;
    lcs[k] = c;
    lsn[k] = sv;
    G[L.cs + k] = c;
    G[L.sn + k] = sv;
    gnext = -sv * gp;
    gk = c * gp;
  };
  double gpj;   // provisional g[j] entry before the rotation of column j
  if (j == 0) {
    // u = r / |r| in the basis precision: |r| alpha is the exact start norm
    if (alpha == 0.0) {
      out[5] = 2.0;
      return;
    }
    gpj = misc[0] * alpha;
    G[L.gpre] = gpj;
  } else {
    // u = (A z_{j-1} - sum_{i<j} h_{i,j-1} v_i) / alpha_{j-1} = sum_{i<j} s_i v_i + alpha v_j
    const double ap = misc[1];
    for (int i = 0; i < j; ++i) colA[i] += ap * dd[i];
    colA[j] = ap * alpha;
    double gk, gn;
    rotate(colA, j - 1, misc[0], gk, gn);
    for (int i = 0; i < j; ++i) G[L.R + i * m + j - 1] = colA[i];
    G[L.g + j - 1] = gk;
    G[L.g + j] = gn;
    G[L.gpre + j] = gn;
    out[3] = gn;
    gpj = gn;
  }
  // provisional column j (subdiagonal beta until step j + 1 completes it)
  for (int i = 0; i < j; ++i) colB[i] = dd[j + 1 + i];
  colB[j] = h;
  colB[j + 1] = beta;
  for (int i = 0; i <= j + 1; ++i) G[L.Hr + i * m + j] = colB[i];
  double gk, gn;
  rotate(colB, j, gpj, gk, gn);
  double* sr = G + L.snapR + (j & 1) * (m + 1);
  for (int i = 0; i <= j; ++i) {
    G[L.R + i * m + j] = colB[i];
    sr[i] = colB[i];
  }
  G[L.g + j] = gk;
  G[L.g + j + 1] = gn;
  G[L.gpre + j + 1] = gn;
  G[L.snapg + (j & 1)] = gk;
  out[4] = gn;
  G[L.ap] = alpha;
}

__global__ void k_givens_solve(const double* __restrict__ G, GivensLayout L, int m, int jn, int snap_j,
                               double* __restrict__ y) {
#pragma clang fp contract(off)
  if (threadIdx.x != 0) return;
  const double *R = G + L.R, *g = G + L.g;
  const double* sr = G + L.snapR + (snap_j >= 0 ? (snap_j & 1) * (m + 1) : 0);
  auto r = [&](int i, int k) { return k == snap_j ? sr[i] : R[i * m + k]; };
  for (int i = jn - 1; i >= 0; --i) {
    double t = i == snap_j ? G[L.snapg + (snap_j & 1)] : g[i];
    for (int k = i + 1; k < jn; ++k) t -= r(i, k) * y[k];
    y[i] = t / r(i, i);
  }
}

// out[g] = sum_q X[g][q] over the Qs values of row g (one block per row).
__global__ void __launch_bounds__(TPB) k_row_sums(const double* __restrict__ X, int64_t Qs, double* __restrict__ out) {
  __shared__ double sh[TPB / 64];
  const double* row = X + static_cast<int64_t>(blockIdx.x) * Qs;
  double v = 0.0;
  for (int64_t q = threadIdx.x; q < Qs; q += blockDim.x) v += row[q];
  const double tot = block_sum(v, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = tot;
}


template <class T>
__global__ void __launch_bounds__(TPB) k_multidot(const T* __restrict__ V, int64_t ldv, int k,
                                                  const T* __restrict__ w, int64_t n, double* __restrict__ part) {
  // groups of 8 dot products share one block reduction
  __shared__ double sh[(TPB / 64) * 8];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * RED_CHUNK + threadIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double wr[RED_E];
#pragma unroll
  for (int e = 0; e < RED_E; ++e) {
    const int64_t i = base + static_cast<int64_t>(e) * TPB;
    wr[e] = (i < n) ? static_cast<double>(w[i]) : 0.0;
  }
  for (int jg = 0; jg < k; jg += 8) {
    double acc[8];
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) acc[jj] = 0.0;
#pragma unroll
    for (int e = 0; e < RED_E; ++e) {
      const int64_t i = base + static_cast<int64_t>(e) * TPB;
      if (i < n) {
#pragma unroll
        for (int jj = 0; jj < 8; ++jj)
          if (jg + jj < k) acc[jj] += static_cast<double>(V[static_cast<int64_t>(jg + jj) * ldv + i]) * wr[e];
      }
    }
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) acc[jj] = wave_sum(acc[jj]);
    __syncthreads();
    if (lane == 0)
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) sh[wv * 8 + jj] = acc[jj];
    __syncthreads();
    if (threadIdx.x < 8 && jg + static_cast<int>(threadIdx.x) < k) {
      double s = 0.0;
      for (int q = 0; q < (TPB / 64); ++q) s += sh[q * 8 + threadIdx.x];
      part[static_cast<int64_t>(blockIdx.x) * k + jg + threadIdx.x] = s;
    }
  }
}


// Vector-load variant (16-byte aligned columns): loads are clamped and
// unconditional so a thread issues all of them before accumulating.  The
// n % VEC trailing elements are added by the first threads of block 0.
template <class T, int VEC>
__global__ void __launch_bounds__(TPB) k_multidot_v(const T* __restrict__ V, int64_t ldv, int k,
                                                    const T* __restrict__ w, int64_t n, double* __restrict__ part) {
  __shared__ double sh[(TPB / 64) * 8];
  constexpr int NV = RED_E / VEC;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * RED_CHUNK + static_cast<int64_t>(threadIdx.x) * VEC;
  const int64_t nv = n - n % VEC;
  const int64_t it = nv + threadIdx.x;   // tail element of this thread (block 0)
  const bool tail = blockIdx.x == 0 && it < n;
  const double wt = tail ? static_cast<double>(w[it]) : 0.0;
  double wr[NV][VEC];
  int64_t ic[NV];
#pragma unroll
  for (int e = 0; e < NV; ++e) {
    const int64_t i = base + static_cast<int64_t>(e) * TPB * VEC;
    const bool ok = i < nv;
    ic[e] = ok ? i : 0;
    double t[VEC];
    loadv<VEC, T, double>(w + ic[e], t);
#pragma unroll
    for (int q = 0; q < VEC; ++q) wr[e][q] = ok ? t[q] : 0.0;
  }
  for (int jg = 0; jg < k; jg += 8) {
    double acc[8];
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) acc[jj] = 0.0;
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
      const int jv = min(jg + jj, k - 1);
      const T* Vj = V + static_cast<int64_t>(jv) * ldv;
#pragma unroll
      for (int e = 0; e < NV; ++e) {
        double t[VEC];
        loadv<VEC, T, double>(Vj + ic[e], t);
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc[jj] += t[q] * wr[e][q];
      }
      if (tail) acc[jj] += static_cast<double>(Vj[it]) * wt;
    }
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) acc[jj] = wave_sum(acc[jj]);
    __syncthreads();
    if (lane == 0)
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) sh[wv * 8 + jj] = acc[jj];
    __syncthreads();
    if (threadIdx.x < 8 && jg + static_cast<int>(threadIdx.x) < k) {
      double s = 0.0;
      for (int q = 0; q < (TPB / 64); ++q) s += sh[q * 8 + threadIdx.x];
      part[static_cast<int64_t>(blockIdx.x) * k + jg + threadIdx.x] = s;
    }
  }
}

// Two right-hand sides in one pass over V: partial sums of V_i . a and
// V_i . b (i < k) into part[blk][2k] = {V_i . a ..., V_i . b ...}.  a and b
// are kept in registers in their storage type; products and sums are FP64.
template <class T, int VEC>
__global__ void __launch_bounds__(TPB) k_multidot2(const T* __restrict__ V, int64_t ldv, int k,
                                                   const T* __restrict__ a, const T* __restrict__ b, int64_t n,
                                                   double* __restrict__ part) {
  __shared__ double sh[(TPB / 64) * 8];
  constexpr int NV = RED_E / VEC;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * RED_CHUNK + static_cast<int64_t>(threadIdx.x) * VEC;
  const int64_t nv = n - n % VEC;
  const int64_t it = nv + threadIdx.x;   // tail element of this thread (block 0)
  const bool tail = blockIdx.x == 0 && it < n;
  const double at = tail ? static_cast<double>(a[it]) : 0.0;
  const double bt = tail ? static_cast<double>(b[it]) : 0.0;
  T ar[NV][VEC], br[NV][VEC];
  int64_t ic[NV];
#pragma unroll
  for (int e = 0; e < NV; ++e) {
    const int64_t i = base + static_cast<int64_t>(e) * TPB * VEC;
    const bool ok = i < nv;
    ic[e] = ok ? i : 0;
    loadv<VEC, T, T>(a + ic[e], ar[e]);
    loadv<VEC, T, T>(b + ic[e], br[e]);
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
      if (!ok) ar[e][q] = T(0);
      if (!ok) br[e][q] = T(0);
    }
  }
  for (int jg = 0; jg < k; jg += 4) {
    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int jv = min(jg + jj, k - 1);
      const T* Vj = V + static_cast<int64_t>(jv) * ldv;
#pragma unroll
      for (int e = 0; e < NV; ++e) {
        T t[VEC];
        loadv<VEC, T, T>(Vj + ic[e], t);
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
          const double tv = static_cast<double>(t[q]);
          acc[jj] += tv * static_cast<double>(ar[e][q]);
          acc[4 + jj] += tv * static_cast<double>(br[e][q]);
        }
      }
      if (tail) {
        const double tv = static_cast<double>(Vj[it]);
        acc[jj] += tv * at;
        acc[4 + jj] += tv * bt;
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = wave_sum(acc[q]);
    __syncthreads();
    if (lane == 0)
#pragma unroll
      for (int q = 0; q < 8; ++q) sh[wv * 8 + q] = acc[q];
    __syncthreads();
    if (threadIdx.x < 8) {
      const int q = threadIdx.x;
      const int col = jg + (q & 3);
      if (col < k) {
        double s = 0.0;
        for (int w = 0; w < (TPB / 64); ++w) s += sh[w * 8 + q];
        part[static_cast<int64_t>(blockIdx.x) * 2 * k + (q >= 4 ? k : 0) + col] = s;
      }
    }
  }
}

// One Arnoldi step's Gram-Schmidt with the second pass of the previous
// vector merged in.  Column j of V holds u (orthogonalized once),
// column j + 1 holds w; dots = {V_i . u (i <= j), V_i . w (i <= j)} from
// k_multidot2 over the j + 1 first columns.  With s_i = V_i . u, t_i = V_i . w
// (i < j), alpha = sqrt(u.u - s.s) and h = (u.w - s.t) / alpha, it writes
//   v = (u - sum_i s_i V_i) / alpha          into column j  (u made orthonormal),
//   w' = (w - sum_i t_i V_i - h v) / alpha   into column j + 1,
// the partial sums of |w'|^2 into part, and {alpha, h} into sc (block 0).
// The division of w' by alpha keeps the basis vectors of order one: w scales
// with u, and u with the previous w', so unscaled norms would multiply along
// a restart cycle.  alpha is 0 when u.u - s.s <= 0 (u numerically in the
// span of V); v and w' are then 0.
template <class T>
__global__ void __launch_bounds__(TPB) k_dcgs_update(T* __restrict__ V, int64_t ldv, int j,
                                                     const double* __restrict__ dots, int64_t n,
                                                     double* __restrict__ part, double* __restrict__ sc) {
  __shared__ double sh[TPB / 64];
  __shared__ double ss[64], ts[64], hs[3];
  const int k = j + 1;
  for (int i = threadIdx.x; i < j; i += TPB) {
    ss[i] = dots[i];
    ts[i] = dots[k + i];
  }
  if (threadIdx.x == 0) {
    double s2 = 0.0, st = 0.0;
    for (int i = 0; i < j; ++i) {
      s2 += dots[i] * dots[i];
      st += dots[i] * dots[k + i];
    }
    const double a2 = dots[j] - s2;
    const double al = a2 > 0.0 ? sqrt(a2) : 0.0;
    const double inv = al > 0.0 ? 1.0 / al : 0.0;
    hs[0] = al;
    hs[1] = (dots[k + j] - st) * inv;
    hs[2] = inv;
    if (blockIdx.x == 0) {
      sc[0] = hs[0];
      sc[1] = hs[1];
    }
  }
  __syncthreads();
  const double h = hs[1], inv = hs[2];
  T* u = V + static_cast<int64_t>(j) * ldv;
  T* w = u + ldv;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * RED_CHUNK + threadIdx.x;
  double acc = 0.0;
  for (int e = 0; e < RED_E; ++e) {
    const int64_t i = base + static_cast<int64_t>(e) * TPB;
    if (i >= n) break;
    double pv = 0.0, pw = 0.0;
    for (int l = 0; l < j; ++l) {
      const double vl = static_cast<double>(V[static_cast<int64_t>(l) * ldv + i]);
      pv += ss[l] * vl;
      pw += ts[l] * vl;
    }
    const T vt = static_cast<T>((static_cast<double>(u[i]) - pv) * inv);
    u[i] = vt;
    const T wt = static_cast<T>((static_cast<double>(w[i]) - pw - h * static_cast<double>(vt)) * inv);
    w[i] = wt;
    acc += static_cast<double>(wt) * static_cast<double>(wt);
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(TPB) k_finalize_sum(const double* __restrict__ part, int nb, int k,
                                                      double* __restrict__ out) {
  __shared__ double sh[TPB / 64];
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += TPB) acc += part[static_cast<int64_t>(b) * k + j];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) out[j] = s;
}

// out[q] = max_b part[2 b + q], q = 0, 1 (one block per q)
__global__ void __launch_bounds__(TPB) k_finalize_max2(const double* __restrict__ part, int64_t nb, double* __restrict__ out) {
  __shared__ double sh[TPB / 64];
  double m = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += TPB) m = fmax(m, part[2 * b + blockIdx.x]);
  const double s = block_max(m, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ void __launch_bounds__(TPB) k_finalize_max(const double* __restrict__ part, int nb, double* __restrict__ out) {
  __shared__ double sh[TPB / 64];
  double m = 0.0;
  for (int b = threadIdx.x; b < nb; b += TPB) m = fmax(m, part[b]);
  const double s = block_max(m, sh);
  if (threadIdx.x == 0) out[0] = s;
}

template <class T>
__global__ void __launch_bounds__(TPB) k_update_norm(const T* __restrict__ V, int64_t ldv, int k,
                                                     const double* __restrict__ h, T* __restrict__ w, int64_t n,
                                                     double* __restrict__ part) {
  __shared__ double sh[TPB / 64];
  __shared__ double hs[128];
  for (int j = threadIdx.x; j < k; j += TPB) hs[j] = h[j];
  __syncthreads();
  const int64_t base = static_cast<int64_t>(blockIdx.x) * RED_CHUNK + threadIdx.x;
  double acc = 0.0;
  for (int e = 0; e < RED_E; ++e) {
    const int64_t i = base + static_cast<int64_t>(e) * TPB;
    if (i >= n) break;
    double v = static_cast<double>(w[i]);
    for (int j = 0; j < k; ++j) v -= hs[j] * static_cast<double>(V[static_cast<int64_t>(j) * ldv + i]);
    const T vt = static_cast<T>(v);
    w[i] = vt;
    acc += static_cast<double>(vt) * static_cast<double>(vt);
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(TPB) k_absmax(const double* __restrict__ x, int64_t n, double* __restrict__ part) {
  __shared__ double sh[TPB / 64];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * RED_CHUNK + threadIdx.x;
  double m = 0.0;
  for (int e = 0; e < RED_E; ++e) {
    const int64_t i = base + static_cast<int64_t>(e) * TPB;
    if (i < n) m = fmax(m, fabs(x[i]));
  }
  const double s = block_max(m, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(TPB) k_sumsq(const double* __restrict__ x, int64_t n, double* __restrict__ part) {
  __shared__ double sh[TPB / 64];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * RED_CHUNK + threadIdx.x;
  double acc = 0.0;
  for (int e = 0; e < RED_E; ++e) {
    const int64_t i = base + static_cast<int64_t>(e) * TPB;
    if (i < n) acc += x[i] * x[i];
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// ---------------------------------------------------------------- vector ops
template <class T>
__global__ void k_scale_by_dev(T* __restrict__ x, int64_t n, const double* __restrict__ nrm2) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] = static_cast<T>(static_cast<double>(x[i]) * (1.0 / sqrt(nrm2[0])));
}
// Shock-capturing coefficient from omega |R| at the Gauss points of one
// linearization: R[g][q] *= fac[g] / den with den = Cm (max|u| / T + max|u_t|)
// from the device maxima (maxes[0], maxes[1]); zero when den is 0.
__global__ void k_sc_scale(double* __restrict__ R, const double* __restrict__ fac, const double* __restrict__ maxes,
                           double Cm, double invT, int64_t Qs, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double den = Cm * (maxes[0] * invT + maxes[1]);
  R[i] = den > 0.0 ? R[i] * fac[i / Qs] / den : 0.0;
}
// y = a * x (FP64 in, basis type out)
template <class T>
__global__ void k_scale_to(const double* __restrict__ x, double a, T* __restrict__ y, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = static_cast<T>(a * x[i]);
}
// r = b - y (y in basis type)
template <class T>
__global__ void k_sub_from(const double* __restrict__ b, const T* __restrict__ y, double* __restrict__ r, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) r[i] = b[i] - static_cast<double>(y[i]);
}
__global__ void k_axpby(double a, const double* __restrict__ x, double b, double* __restrict__ y, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}
template <class T>
__global__ void k_combine(const T* __restrict__ Z, int64_t ldz, int k, const double* __restrict__ c,
                          double* __restrict__ x, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = x[i];
  for (int j = 0; j < k; ++j) v += c[j] * static_cast<double>(Z[static_cast<int64_t>(j) * ldz + i]);
  x[i] = v;
}
template <class A, class B>
__global__ void k_convert(const A* __restrict__ x, B* __restrict__ y, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = from_c<B>(to_c(x[i], float(0)));
}
__global__ void k_fill(double* __restrict__ x, double v, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}
__global__ void k_add_unknowns(double* __restrict__ u, const double* __restrict__ d, double a, int64_t n, int64_t Ns) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) u[Ns + i] += a * d[i];
}

// ---------------------------------------------------------------- linearization
// f(x, t) of a Source (see kernels.hpp).  Products and sums are rounded one
// by one (no fused multiply-add), so that an indicator decides a point's
// membership from the same rounded distance as a plain evaluation of
// sum_l ((x_l - c_l) - v_l t)^2 in direction order.
__device__ __forceinline__ double source_value(const Source& f, double x0, double x1, double x2, double t) {
  if (!(t >= f.t0 && t <= f.t1)) return 0.0;
  const double x[3] = {x0, x1, x2};
  double r2 = 0.0;
  for (int l = 0; l < f.d; ++l) {
    double dx = __dsub_rn(x[l], f.c[l]);
    if (f.kind == 2) dx = __dsub_rn(dx, __dmul_rn(f.v[l], t));
    r2 = __dadd_rn(r2, __dmul_rn(dx, dx));
  }
  if (f.kind == 1) return r2 <= f.r2 ? f.amp : 0.0;
  return f.amp * exp(-f.kappa * r2);
}

__global__ void __launch_bounds__(TPB) k_pointwise_ionic(
    const double* __restrict__ u, const double* __restrict__ ut, const double* __restrict__ lap,
    const double* __restrict__ w, const double* __restrict__ wt, const double* __restrict__ ws, int64_t Qs,
    int64_t total, double Cm, double a, double c1, double c2, double* __restrict__ g, double* __restrict__ absR,
    double* __restrict__ part, Source f, int q0, int Q1, int Q2, double* __restrict__ Cq, double* __restrict__ Rq) {
  __shared__ double sh[TPB / 64];
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  double mu = 0.0, mt = 0.0;
  if (idx < total) {
    const int64_t qt = idx / Qs, qs = idx - qt * Qs;
    const double uu = u[idx], ww = w[idx], tt = ut[idx];
    double I = c1 * uu * (uu - a) * (uu - 1.0) + c2 * uu * ww;
    if (f.kind) {
      const int q1 = static_cast<int>(qs % Q1);
      const int64_t r = qs / Q1;
      const int q2 = static_cast<int>(r % Q2), q3 = static_cast<int>(r / Q2);
      I -= source_value(f, f.xq[0][q1], f.d > 1 ? f.xq[1][q2] : 0.0, f.d > 2 ? f.xq[2][q3] : 0.0,
                        f.tq[q0 + qt]);
    }
    g[idx] = wt[qt] * ws[qs] * I;
    if (Cq) Cq[static_cast<int64_t>(q0) * Qs + idx] = wt[qt] * ws[qs] * (c1 * (uu - a) * (uu - 1.0) + c2 * ww);
    absR[idx] = fabs(Cm * tt - lap[idx] + I);
    if (Rq) Rq[static_cast<int64_t>(q0) * Qs + idx] = wt[qt] * ws[qs] * absR[idx];
    mu = fabs(uu);
    mt = fabs(tt);
  }
  const double m1 = block_max(mu, sh);
  if (threadIdx.x == 0) part[2 * blockIdx.x] = m1;
  const double m2 = block_max(mt, sh);
  if (threadIdx.x == 0) part[2 * blockIdx.x + 1] = m2;
}

// Quadrature pass fused along the slowest spatial axis (FP64): from the
// arrays expanded along the faster axes (layout [row][nd][Qin], one row per
// time Gauss point) it forms, at every Gauss point of the axis,
//   u = B0 A0,  lap = sL B2 A0 + sM B0 A1 + sF B0 A2,  u_t = B0 UT,  w = B0 WW,
// then I = c1 u (u - a)(u - 1) + c2 u w, |R| = |Cm u_t - lap + I|, and
//   - M[et][e][c]: max of |R| over the Gauss points of space-time element
//     (et, e) in column c (when M is given),
//   - G[row][i][c]: sum over the axis' Gauss points of B0 wt ws I
//     (projection onto the axis' B-splines, when G is given),
//   - block maxima of |u| and |u_t| into part[2 b], part[2 b + 1] (b = boff +
//     linear block index).
// A block has one wave per time Gauss row of time element et (blockIdx.y);
// lane l owns column 64 blockIdx.x + l.  Each thread walks the elements of
// chunk blockIdx.z with rings of the KP input rows an element touches; the
// element maximum over the time rows is taken across the waves through LDS
// (double-buffered, one barrier per element).  With D == 2, A1 is not read.
template <int D, int KP, bool X2>
__global__ void __launch_bounds__(384) k_quad_fused(
    const double* __restrict__ A0, const double* __restrict__ A1, const double* __restrict__ A2,
    const double* __restrict__ UT, const double* __restrict__ WW, int nd, int64_t Qin,
    const double* __restrict__ B0, const double* __restrict__ B2, const int* __restrict__ efirst,
    const int* __restrict__ chunks, const double* __restrict__ wt, const double* __restrict__ win,
    const double* __restrict__ wd, double sL,
    double sM, double sF, double Cm, double a, double c1, double c2, double* __restrict__ G,
    double* __restrict__ M, int nel_d, double* __restrict__ part, int64_t boff, int n2, int Q1,
    const double* __restrict__ e0x2, const double* __restrict__ e2x2, const int* __restrict__ f2x, Source fsrc, int q0,
    double* __restrict__ Cq, double* __restrict__ Rq, int64_t Qs) {
  __shared__ double sh[8];
  __shared__ double smax[2][6][64];
  const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
  const int nqt = blockDim.x >> 6;
  // column blocks, XCD-aware: gridDim.x is a multiple of 8 and workgroups go
  // to the 8 XCDs in turn, so XCD k walks the contiguous column blocks
  // [k gridDim.x / 8, (k + 1) gridDim.x / 8); with X2, neighbouring columns
  // read the same x1-expanded rows and find them in that XCD's L2
  const int64_t lx = static_cast<int64_t>(blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  const int64_t c = lx * 64 + lane;
  const bool cv = c < Qin;
  const int64_t cc = cv ? c : 0;
  const int et = blockIdx.y;
  const int e0 = chunks[4 * blockIdx.z], e1 = chunks[4 * blockIdx.z + 1];
  const int d0 = chunks[4 * blockIdx.z + 2], d1 = chunks[4 * blockIdx.z + 3];
  const int64_t lay = static_cast<int64_t>(nd) * Qin;
  const int tr = et * nqt + row;
  const int64_t rb = static_cast<int64_t>(tr) * lay + cc;
  const double wtr = wt[tr];
  const double wc = win[cc];   // product of the faster axes' Gauss weights of column c
  // source term: coordinates of this thread's column and time row
  double fx0 = 0.0, fx1 = 0.0, ftt = 0.0;
  if (fsrc.kind) {
    ftt = fsrc.tq[q0 + tr];
    if constexpr (D == 3) {
      fx0 = fsrc.xq[0][cc % fsrc.Q1];
      fx1 = fsrc.xq[1][cc / fsrc.Q1];
    } else {
      fx0 = fsrc.xq[0][cc];
    }
  }
  double a0[KP], a1[D == 3 ? KP : 1], a2[KP], ut[KP], ww[KP], gr[KP];
  // X2 (D == 3): the inputs are expanded along x1 only ([row][nd][n2][Q1]:
  // A0 = B0 u, A2 = B2 u along x1, UT, WW) and the x2 expansion is formed
  // here, column c = q1 + Q1 q2 reading rows f2x[q2] + k with the weights
  // e0x2 / e2x2 (values / second derivatives), summed in the order of the
  // x2 gathers it replaces
  int64_t ib = rb, istep = Qin;
  double w0[X2 ? KP : 1], w2[X2 ? KP : 1];
  if constexpr (X2) {
    const int q2 = static_cast<int>(cc / Q1);
    istep = static_cast<int64_t>(n2) * Q1;
    ib = static_cast<int64_t>(tr) * nd * istep + static_cast<int64_t>(f2x[q2]) * Q1 + (cc - static_cast<int64_t>(q2) * Q1);
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      w0[k] = e0x2[q2 * KP + k];
      w2[k] = e2x2[q2 * KP + k];
    }
  }
  auto load = [&](int k, int dof) {
    const bool ok = dof < nd;
    const int64_t o = ib + static_cast<int64_t>(ok ? dof : 0) * istep;
    if constexpr (X2) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
#pragma unroll
      for (int k2 = 0; k2 < KP; ++k2) {
        const int64_t ok2 = o + static_cast<int64_t>(k2) * Q1;
        const double xa = A0[ok2], xb = A2[ok2], xt = UT[ok2], xw = WW[ok2];
        s0 += w0[k2] * xa;
        s1 += w2[k2] * xa;
        s2 += w0[k2] * xb;
        s3 += w0[k2] * xt;
        s4 += w0[k2] * xw;
      }
      a0[k] = ok ? s0 : 0.0;
      if constexpr (D == 3) a1[k] = ok ? s1 : 0.0;
      a2[k] = ok ? s2 : 0.0;
      ut[k] = ok ? s3 : 0.0;
      ww[k] = ok ? s4 : 0.0;
    } else {
      a0[k] = ok ? A0[o] : 0.0;
      if constexpr (D == 3) a1[k] = ok ? A1[o] : 0.0;
      a2[k] = ok ? A2[o] : 0.0;
      ut[k] = ok ? UT[o] : 0.0;
      ww[k] = ok ? WW[o] : 0.0;
    }
    gr[k] = 0.0;
  };
  auto store = [&](int k, int dof) {
    if (G && cv && dof >= d0 && dof < d1 && dof < nd) G[rb + static_cast<int64_t>(dof) * Qin] = gr[k];
  };
  int f = efirst[e0];
#pragma unroll
  for (int k = 0; k < KP; ++k) load(k, f + k);
  double mu = 0.0, mt = 0.0;
  for (int e = e0; e < e1; ++e) {
    const int fn = efirst[e];
    for (; f < fn; ++f) {
      store(0, f);
#pragma unroll
      for (int k = 0; k < KP - 1; ++k) {
        a0[k] = a0[k + 1];
        if constexpr (D == 3) a1[k] = a1[k + 1];
        a2[k] = a2[k + 1];
        ut[k] = ut[k + 1];
        ww[k] = ww[k + 1];
        gr[k] = gr[k + 1];
      }
      load(KP - 1, f + KP);
    }
    double emax = 0.0;
#pragma unroll
    for (int g = 0; g < KP; ++g) {
      const int qd = e * KP + g;
      double u = 0.0, l2 = 0.0, l1 = 0.0, l0 = 0.0, tt = 0.0, w = 0.0;
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        const double b0 = B0[qd * KP + k], b2 = B2[qd * KP + k];
        u += b0 * a0[k];
        l2 += b2 * a0[k];
        if constexpr (D == 3) l1 += b0 * a1[k];
        l0 += b0 * a2[k];
        tt += b0 * ut[k];
        w += b0 * ww[k];
      }
      const double lap = sL * l2 + sM * l1 + sF * l0;
      double I = c1 * u * (u - a) * (u - 1.0) + c2 * u * w;
      if (fsrc.kind) {
        const double xd = fsrc.xq[D - 1][qd];
        I -= (D == 3) ? source_value(fsrc, fx0, fx1, xd, ftt) : source_value(fsrc, fx0, xd, 0.0, ftt);
      }
      const double aR = fabs(Cm * tt - lap + I);
      emax = fmax(emax, aR);
      if (Rq && cv)
        Rq[static_cast<int64_t>(q0 + tr) * Qs + static_cast<int64_t>(qd) * Qin + c] = wtr * (wc * wd[qd]) * aR;
      mu = fmax(mu, fabs(u));
      mt = fmax(mt, fabs(tt));
      const double gv = wtr * (wc * wd[qd]) * I;
      if (Cq && cv)
        Cq[static_cast<int64_t>(q0 + tr) * Qs + static_cast<int64_t>(qd) * Qin + c] =
            wtr * (wc * wd[qd]) * (c1 * (u - a) * (u - 1.0) + c2 * w);
#pragma unroll
      for (int k = 0; k < KP; ++k) gr[k] += B0[qd * KP + k] * gv;
    }
    if (M) {
      smax[e & 1][row][lane] = emax;
      __syncthreads();
      if (row == 0 && cv) {
        double m = smax[e & 1][0][lane];
        for (int r = 1; r < nqt; ++r) m = fmax(m, smax[e & 1][r][lane]);
        M[(static_cast<int64_t>(et) * nel_d + e) * Qin + c] = m;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < KP; ++k) store(k, f + k);
  if (!cv) mu = mt = 0.0;
  const int64_t b = boff + blockIdx.x + static_cast<int64_t>(gridDim.x) * (blockIdx.y + static_cast<int64_t>(gridDim.y) * blockIdx.z);
  const double m1 = block_max(mu, sh);
  if (threadIdx.x == 0) part[2 * b] = m1;
  const double m2 = block_max(mt, sh);
  if (threadIdx.x == 0) part[2 * b + 1] = m2;
}

__global__ void k_theta_finish(double* __restrict__ th, int64_t n, const double* __restrict__ maxes, double Cm,
                               double invT) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double den = Cm * (maxes[0] * invT + maxes[1]);
  const double num = th[i];
  th[i] = (den > 0.0) ? fmin(num / den, 1.0) : (num > 0.0 ? 1.0 : 0.0);
}

__global__ void k_react_grid(const double* __restrict__ u, const double* __restrict__ w, double* __restrict__ c,
                             int64_t n, double a, double c1, double c2, int newton) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double uu = u[i], ww = w[i];
  c[i] = newton ? c1 * (3.0 * uu * uu - 2.0 * (1.0 + a) * uu + a) + c2 * ww
                : c1 * (uu - a) * (uu - 1.0) + c2 * ww;
}

// Gram partials: block b accumulates C[:, cols] C[:, cols]^T over its column chunks.
constexpr int GRAM_CH = 32;
constexpr int GRAM_MAXE = 40;   // entries per thread (m(m+1)/2 <= 40*256)
__global__ void __launch_bounds__(TPB) k_gram(const double* __restrict__ C, int m, int64_t n,
                                              double* __restrict__ part) {
  extern __shared__ char smem_raw[];
  double* tile = reinterpret_cast<double*>(smem_raw);   // [m][GRAM_CH]
  const int ne = m * (m + 1) / 2;
  double acc[GRAM_MAXE];
  int ei[GRAM_MAXE], ej[GRAM_MAXE];
#pragma unroll
  for (int k = 0; k < GRAM_MAXE; ++k) {
    acc[k] = 0.0;
    int e = threadIdx.x + k * TPB;
    int i = 0;
    if (e < ne) {   // e -> (i, j), j >= i, row-major over the upper triangle
      int rem = e;
      while (rem >= m - i) { rem -= m - i; ++i; }
      ei[k] = i;
      ej[k] = i + rem;
    } else {
      ei[k] = -1;
      ej[k] = -1;
    }
  }
  const int64_t nch = (n + GRAM_CH - 1) / GRAM_CH;
  for (int64_t ch = blockIdx.x; ch < nch; ch += gridDim.x) {
    __syncthreads();
    for (int t = threadIdx.x; t < m * GRAM_CH; t += TPB) {
      const int i = t / GRAM_CH, c = t % GRAM_CH;
      const int64_t col = ch * GRAM_CH + c;
      tile[t] = (col < n) ? C[static_cast<int64_t>(i) * n + col] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < GRAM_MAXE; ++k) {
      if (ei[k] < 0) continue;
      const double* a = tile + ei[k] * GRAM_CH;
      const double* b = tile + ej[k] * GRAM_CH;
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < GRAM_CH; ++c) s += a[c] * b[c];
      acc[k] += s;
    }
  }
  const int64_t mm = static_cast<int64_t>(m) * m;
#pragma unroll
  for (int k = 0; k < GRAM_MAXE; ++k) {
    if (ei[k] < 0) continue;
    part[blockIdx.x * mm + static_cast<int64_t>(ei[k]) * m + ej[k]] = acc[k];
    part[blockIdx.x * mm + static_cast<int64_t>(ej[k]) * m + ei[k]] = acc[k];
  }
}

__global__ void k_right_factor(const double* __restrict__ C, int m, int64_t n, const double* __restrict__ U,
                               const double* __restrict__ inv_s, int R, double* __restrict__ V) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  for (int r = 0; r < R; ++r) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += C[static_cast<int64_t>(i) * n + j] * U[i * R + r];
    V[j * R + r] = s * inv_s[r];
  }
}

__global__ void k_scale_rows(double* __restrict__ P, int64_t total, int64_t Qs, const double* __restrict__ wq) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < total) P[i] *= wq[i % Qs];
}

__global__ void k_transpose_nr(const double* __restrict__ V, int64_t N, int R, double* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N * R) return;
  const int64_t r = i / N, j = i - r * N;
  out[i] = V[j * R + r];
}

}  // namespace

// ======================================================================= wrappers
template <class Ti, class To, class C>
void gather(const DTable<C>& t, const Ti* x, To* y, int64_t outer, int64_t inner, int n_in, int in_base, C alpha,
            C beta, hipStream_t s) {
  const int64_t total = outer * t.n_out * inner;
  if (total == 0) return;
  const double gbytes = static_cast<double>(outer) * n_in * inner * sizeof(Ti) +
                        static_cast<double>(total) * sizeof(To) * (beta != C(0) ? 2 : 1);
  const int64_t nrows = outer * t.n_out;
  const int vec = (inner % 4 == 0) ? 4 : (inner % 2 == 0 ? 2 : 1);
  const bool sweep_w = t.W == 2 || t.W == 3 || t.W == 4 || t.W == 5 || t.W == 7 || t.W == 9 || t.W == 16;
  if (std::is_same<Ti, To>::value && t.c0 != nullptr && sweep_w && inner >= 32 &&
      !(vec == 4 && (reinterpret_cast<uintptr_t>(x) % (4 * sizeof(Ti))) == 0 &&
        (reinterpret_cast<uintptr_t>(y) % (4 * sizeof(To))) == 0)) {
    // inner not a multiple of 4 (or unaligned): flattened columns, E per lane
    const int64_t ncols = outer * inner;
    const int E = 4;
    const int64_t groups = (ncols + 64 * E - 1) / (64 * E);
    const int64_t want = 1 << 12;   // waves
    int64_t nchunks = std::max<int64_t>(1, std::min<int64_t>(t.n_out / 4 + 1, (want + groups - 1) / groups));
    const int rc = static_cast<int>((t.n_out + nchunks - 1) / nchunks);
    nchunks = (t.n_out + rc - 1) / rc;
    const int64_t waves = groups * nchunks;
    ProfScope ps(t_gather_cls, 10 + 32 * prec_code<Ti>(), s, gbytes);
    const unsigned blocks = static_cast<unsigned>((waves * 64 + TPB - 1) / TPB);
#define SF(w)                                                                                                        \
  hipLaunchKernelGGL((k_sweep_flat<Ti, C, w, 4>), dim3(blocks), dim3(TPB), 0, s, t.c0, t.coef, t.n_out, x,              \
                     reinterpret_cast<Ti*>(y), inner, n_in, in_base, alpha, beta, ncols, rc, static_cast<int>(nchunks))
    switch (t.W) {
      case 2: SF(2); break;
      case 3: SF(3); break;
      case 4: SF(4); break;
      case 5: SF(5); break;
      case 7: SF(7); break;
      case 9: SF(9); break;
      default: SF(16); break;
    }
#undef SF
    return;
  }
  if (std::is_same<Ti, To>::value && t.c0 != nullptr && inner >= 2 && inner < (static_cast<int64_t>(1) << 31) &&
      sweep_w &&
      (reinterpret_cast<uintptr_t>(x) % (vec * sizeof(Ti))) == 0 && (reinterpret_cast<uintptr_t>(y) % (vec * sizeof(To))) == 0) {
    const int64_t slots = inner / vec;
    // enough threads to fill the chip: chunk the output rows
    const int64_t want = 1 << 18;
    int64_t nchunks = std::max<int64_t>(1, std::min<int64_t>(t.n_out / 4 + 1, (want + outer * slots - 1) / (outer * slots)));
    const int rc = static_cast<int>((t.n_out + nchunks - 1) / nchunks);
    nchunks = (t.n_out + rc - 1) / rc;
    const int64_t total_t = outer * nchunks * slots;
    if (total_t < (static_cast<int64_t>(1) << 32)) {
      ProfScope ps(t_gather_cls, 10 + 32 * prec_code<Ti>(), s, gbytes);
      const unsigned blocks = static_cast<unsigned>((total_t + TPB - 1) / TPB);
#define SW(w, v)                                                                                                    \
  hipLaunchKernelGGL((k_sweep<Ti, C, w, v>), dim3(blocks), dim3(TPB), 0, s, t.c0, t.coef, t.n_out, x,                \
                     reinterpret_cast<Ti*>(y), static_cast<uint32_t>(inner), n_in, in_base, alpha, beta,             \
                     static_cast<uint32_t>(slots), rc, static_cast<uint32_t>(nchunks), static_cast<uint32_t>(total_t))
#define SWW(v)                  \
  switch (t.W) {                \
    case 2: SW(2, v); break;    \
    case 3: SW(3, v); break;    \
    case 4: SW(4, v); break;    \
    case 5: SW(5, v); break;    \
    case 7: SW(7, v); break;    \
    case 9: SW(9, v); break;    \
    default: SW(16, v); break;  \
  }
      if (vec == 4) { SWW(4) } else if (vec == 2) { SWW(2) } else { SWW(1) }
#undef SWW
#undef SW
      return;
    }
  }
  if (std::is_same<Ti, To>::value && vec > 1 && inner < (static_cast<int64_t>(1) << 31) &&
      (reinterpret_cast<uintptr_t>(x) % (vec * sizeof(Ti))) == 0 && (reinterpret_cast<uintptr_t>(y) % (vec * sizeof(To))) == 0) {
    const int64_t slots = inner / vec;
    const int64_t rpb = slots < TPB ? TPB / slots : 1;
    const int64_t kchunks = rpb > 1 ? 1 : (slots + TPB - 1) / TPB;
    const int64_t blocks = rpb > 1 ? (nrows + rpb - 1) / rpb : kchunks * nrows;
    if (blocks < (static_cast<int64_t>(1) << 31) && nrows < (static_cast<int64_t>(1) << 32)) {
      ProfScope ps(t_gather_cls, 1 + 32 * prec_code<Ti>(), s, gbytes);
#define GV(wc, v)                                                                                              \
  hipLaunchKernelGGL((k_gather_v4<Ti, C, wc, v>), dim3(static_cast<unsigned>(blocks)), dim3(TPB), 0, s, t.col, t.coef, \
                     t.W, t.n_out, x, reinterpret_cast<Ti*>(y), static_cast<uint32_t>(inner), n_in, in_base, alpha,  \
                     beta, static_cast<uint32_t>(nrows), static_cast<uint32_t>(slots), static_cast<uint32_t>(rpb),   \
                     static_cast<uint32_t>(kchunks))
#define GVW(v)                  \
  switch (t.W) {                \
    case 2: GV(2, v); break;    \
    case 3: GV(3, v); break;    \
    case 4: GV(4, v); break;    \
    case 5: GV(5, v); break;    \
    case 7: GV(7, v); break;    \
    case 9: GV(9, v); break;    \
    case 16: GV(16, v); break;  \
    default: GV(0, v); break;   \
  }
      if (vec == 4) { GVW(4) } else { GVW(2) }
#undef GVW
#undef GV
      return;
    }
  }
  if (inner == 1 && std::is_same<Ti, To>::value) {
    // rows per group: about 4096 staged input values, a multiple of 4 rows
    // (the group spans then stay 16-byte aligned)
    int RB = std::max(1, std::min(256, 4096 / std::max(n_in, 1)));
    if (RB >= 4) RB &= ~3;
    const size_t tab = (static_cast<size_t>(t.n_out) * t.W * (sizeof(C) + sizeof(int)) + 15) & ~static_cast<size_t>(15);
    const size_t sh = tab + static_cast<size_t>(RB) * n_in * sizeof(Ti);
    const int64_t groups = (outer + RB - 1) / RB;
    if (sh <= 64 * 1024) {
      ProfScope ps(t_gather_cls, 2 + 32 * prec_code<Ti>(), s, gbytes);
      const int64_t blocks = std::min<int64_t>(groups, 2048);
#define GR(wt) hipLaunchKernelGGL((k_gather_rows<Ti, C, wt>), dim3(static_cast<unsigned>(blocks)), dim3(TPB), sh, s, t.col, t.coef, t.W, t.n_out, x, reinterpret_cast<Ti*>(y), n_in, in_base, alpha, beta, outer, RB)
      switch (t.W) {
        case 3: GR(3); break;
        case 4: GR(4); break;
        case 5: GR(5); break;
        case 7: GR(7); break;
        case 9: GR(9); break;
        case 16: GR(16); break;
        default: GR(0); break;
      }
#undef GR
      return;
    }
  }
  ProfScope ps(t_gather_cls, 0 + 32 * prec_code<Ti>(), s, gbytes);
  if (total < (static_cast<int64_t>(1) << 32))
    hipLaunchKernelGGL((k_gather<Ti, To, C, uint32_t>), dim3(grid_for(total)), dim3(TPB), 0, s, t.col, t.coef, t.W,
                       t.n_out, x, y, static_cast<uint32_t>(inner), n_in, in_base, alpha, beta,
                       static_cast<uint32_t>(total));
  else
    hipLaunchKernelGGL((k_gather<Ti, To, C, int64_t>), dim3(grid_for(total)), dim3(TPB), 0, s, t.col, t.coef, t.W,
                       t.n_out, x, y, inner, n_in, in_base, alpha, beta, total);
}

template <class S, class C>
bool gather_dual(const DTable<C>& P, const DTable<C>& Q, const S* x, const S* z, S* out1, S* out2, int64_t outer,
                 int64_t inner, int n_in, int in_base, C alpha, C beta, hipStream_t s) {
  if (P.c0 == nullptr || P.W != Q.W || P.n_out != Q.n_out || inner < 2) return false;
  const int W = P.W;
  if (!(W == 2 || W == 3 || W == 4 || W == 5 || W == 7 || W == 9 || W == 11)) return false;
  const int64_t ncols = outer * inner;
  if (ncols == 0) return true;
  constexpr int E = 4;
  const int64_t groups = (ncols + 64 * E - 1) / (64 * E);
  const int64_t want = 1 << 12;   // waves
  int64_t nchunks = std::max<int64_t>(1, std::min<int64_t>(P.n_out / 4 + 1, (want + groups - 1) / groups));
  const int rc = static_cast<int>((P.n_out + nchunks - 1) / nchunks);
  nchunks = (P.n_out + rc - 1) / rc;
  const int64_t waves = groups * nchunks;
  const double by = (2.0 * outer * n_in * inner + (out1 ? 2.0 : 1.0) * outer * P.n_out * inner) * sizeof(S);
  ProfScope ps(t_gather_cls, 13 + 32 * prec_code<S>(), s, by);
  const unsigned blocks = static_cast<unsigned>((waves * 64 + TPB - 1) / TPB);
#define SD(w)                                                                                                      \
  hipLaunchKernelGGL((k_sweep_dual<S, C, w, E>), dim3(blocks), dim3(TPB), 0, s, P.c0, P.coef, Q.coef, P.n_out, x, z, \
                     out1, out2, inner, n_in, in_base, alpha, beta, ncols, rc, static_cast<int>(nchunks))
  switch (W) {
    case 2: SD(2); break;
    case 3: SD(3); break;
    case 4: SD(4); break;
    case 5: SD(5); break;
    case 7: SD(7); break;
    case 9: SD(9); break;
    default: SD(11); break;
  }
#undef SD
  return true;
}

template <class Ti, class To, class C>
void gather_rows(const DTable<C>& t, int r0, int nr, const Ti* x, To* y, int64_t outer, int64_t inner, int n_in,
                 int in_base, C alpha, C beta, hipStream_t s) {
  DTable<C> u;
  u.col = t.col + static_cast<int64_t>(r0) * t.W;
  u.coef = t.coef + static_cast<int64_t>(r0) * t.W;
  u.c0 = t.c0 ? t.c0 + r0 : nullptr;
  u.W = t.W;
  u.n_out = nr;
  gather<Ti, To, C>(u, x, y, outer, inner, n_in, in_base, alpha, beta, s);
}

void mode_max(const int* start, const int* cnt, int n_out, const double* x, double* y, int64_t outer, int64_t inner,
              int n_in, hipStream_t s) {
  const int64_t total = outer * n_out * inner;
  if (total == 0) return;
  ProfScope ps(K_MAX, 9, s, static_cast<double>(outer) * (n_in + n_out) * inner * sizeof(double));
  hipLaunchKernelGGL(k_mode_max, dim3(grid_for(total)), dim3(TPB), 0, s, start, cnt, n_out, x, y, inner, n_in, total);
}

template <class S, class C>
void react_point(const S* Z, int nl, int lo_full, const DTable<C>& Bt, const C* Bv, const C* Bd, const int* re0,
                 const int* re1, const C* Cq, const C* Rq, int64_t Qs, int t0, int t1, int p, S* out, C beta,
                 hipStream_t s) {
  const int rows = t1 - t0;
  const int64_t total = static_cast<int64_t>(rows) * Qs;
  if (total == 0 || (!Cq && !Rq)) return;
  if (!Bv) Bv = Bt.coef;
  const int nterm = (Cq ? 1 : 0) + (Rq ? 1 : 0);
  // algorithmic bytes: the input layers, the coefficients at the slab's time
  // Gauss points and the output rows, each once
  ProfScope ps(K_TIME_MIX, 15 + 32 * prec_code<S>(), s,
               (static_cast<double>(nl) + rows) * Qs * sizeof(S) +
                   nterm * static_cast<double>(rows) * (p + 1) * Qs * sizeof(C),
               nterm * 2.0 * (p + 1) * (p + 1) * (p + 2) * static_cast<double>(total));
  const dim3 g(grid_for(total)), b(TPB);
#define RP(KP_) hipLaunchKernelGGL((k_react_point<S, C, KP_>), g, b, 0, s, Z, nl, lo_full, Bt.coef, Bv, Bd, Bt.c0, \
                                   re0, re1, Cq, Rq, Qs, t0, rows, out, beta)
  switch (p) {
    case 1: RP(2); break;
    case 2: RP(3); break;
    case 3: RP(4); break;
    case 4: RP(5); break;
    default: RP(6); break;
  }
#undef RP
}

bool band_factor(const double* A, const double* B, int Nt, const double* lam, double shift, int64_t Ns, int p,
                 double* F, hipStream_t s) {
  if (Ns == 0) return true;
  const dim3 g(grid_for(Ns)), b(TPB);
  switch (p) {
    case 1: hipLaunchKernelGGL(k_band_factor<1>, g, b, 0, s, A, B, Nt, lam, shift, Ns, F); break;
    case 2: hipLaunchKernelGGL(k_band_factor<2>, g, b, 0, s, A, B, Nt, lam, shift, Ns, F); break;
    case 3: hipLaunchKernelGGL(k_band_factor<3>, g, b, 0, s, A, B, Nt, lam, shift, Ns, F); break;
    case 4: hipLaunchKernelGGL(k_band_factor<4>, g, b, 0, s, A, B, Nt, lam, shift, Ns, F); break;
    case 5: hipLaunchKernelGGL(k_band_factor<5>, g, b, 0, s, A, B, Nt, lam, shift, Ns, F); break;
    default: return false;
  }
  return true;
}

template <class S, class C>
bool band_solve(const C* F, int Nt, int64_t Ns, int p, const S* r, S* x, hipStream_t s) {
  if (Ns == 0) return true;
  // algorithmic bytes: r read, x written, x read back and written, the factors read
  ProfScope ps(K_ARROW, 16 + 32 * prec_code<S>(), s,
               static_cast<double>(Nt) * Ns * (4.0 * sizeof(S) + (2.0 * p + 1.0) * sizeof(C)),
               static_cast<double>(Nt) * Ns * (4.0 * p + 1.0));
  const dim3 g(grid_for(Ns)), b(TPB);
  switch (p) {
    case 1: hipLaunchKernelGGL((k_band_solve<S, C, 1>), g, b, 0, s, F, Nt, Ns, r, x); break;
    case 2: hipLaunchKernelGGL((k_band_solve<S, C, 2>), g, b, 0, s, F, Nt, Ns, r, x); break;
    case 3: hipLaunchKernelGGL((k_band_solve<S, C, 3>), g, b, 0, s, F, Nt, Ns, r, x); break;
    case 4: hipLaunchKernelGGL((k_band_solve<S, C, 4>), g, b, 0, s, F, Nt, Ns, r, x); break;
    case 5: hipLaunchKernelGGL((k_band_solve<S, C, 5>), g, b, 0, s, F, Nt, Ns, r, x); break;
    default: return false;
  }
  return true;
}

void row_sums(const double* X, int rows, int64_t Qs, double* out, hipStream_t s) {
  if (rows > 0) hipLaunchKernelGGL(k_row_sums, dim3(rows), dim3(TPB), 0, s, X, Qs, out);
}

template <class S, class C>
void time_mix(const C* T, const S* Psi, int r0, int r1, int Nt, int t0, int t1, int p, const S* Z, int n_in,
              int in_base, S* out, int64_t Qs, hipStream_t s) {
  const int R = r1 - r0;
  int tpb = TPB;
  while (tpb > 64 && static_cast<size_t>(R) * tpb * sizeof(C) > 64 * 1024) tpb /= 2;
  const size_t sh = static_cast<size_t>(R > 0 ? R : 1) * tpb * sizeof(C);
  const dim3 g(grid_for(Qs, tpb)), b(tpb);
  ProfScope ps(K_TIME_MIX, 3 + 32 * prec_code<S>(), s, (static_cast<double>(n_in) + R + (t1 - t0)) * Qs * sizeof(S),
               2.0 * R * (2 * p + 2) * static_cast<double>(t1 - t0) * Qs);
  switch (p) {
    case 1: hipLaunchKernelGGL((k_time_mix<S, C, 1>), g, b, sh, s, T, Psi, r0, R, Nt, t0, t1, Z, n_in, in_base, out, Qs); break;
    case 2: hipLaunchKernelGGL((k_time_mix<S, C, 2>), g, b, sh, s, T, Psi, r0, R, Nt, t0, t1, Z, n_in, in_base, out, Qs); break;
    case 3: hipLaunchKernelGGL((k_time_mix<S, C, 3>), g, b, sh, s, T, Psi, r0, R, Nt, t0, t1, Z, n_in, in_base, out, Qs); break;
    case 4: hipLaunchKernelGGL((k_time_mix<S, C, 4>), g, b, sh, s, T, Psi, r0, R, Nt, t0, t1, Z, n_in, in_base, out, Qs); break;
    default: hipLaunchKernelGGL((k_time_mix<S, C, 5>), g, b, sh, s, T, Psi, r0, R, Nt, t0, t1, Z, n_in, in_base, out, Qs); break;
  }
}

template <class S, class C>
bool coef_fused(const C* T, const S* Psi, int r0, int r1, int Nt, int t0, int t1, int pt, int ps, const S* Z,
                int n_in, int in_base, const C* Bl, const int* efirst, const int* chunks, int nchunk, int nd,
                int64_t Qin, S* out, int64_t Qs, hipStream_t s) {
  // output rows per thread: 8 in FP32, 4 in FP64 (register rings of the same size)
  constexpr int TS = std::is_same<C, double>::value ? 4 : 8;
  constexpr bool f64 = std::is_same<C, double>::value;
  if (pt < 1 || pt > 5 || ps < 1 || ps > 4) return false;
  if (t1 <= t0 || Qin == 0) return true;
  const int R = r1 - r0;
  const int nslab = (t1 - t0 + TS - 1) / TS;
  const int64_t ncb = (Qin + TPB - 1) / TPB;
  const dim3 g(static_cast<unsigned>((ncb * nchunk + 7) / 8 * 8 * nslab));
  const double rows = static_cast<double>(t1 - t0);
  // algorithmic flops per output row and Gauss point: the time mixing
  // (2 R (2 p_t + 2)) plus the expansion and projection along the axis (4 (p_s + 1))
  const double fl = rows * static_cast<double>(Qs) * (2.0 * R * (2 * pt + 2) + 4.0 * (ps + 1));
  // 32-bit element indices when every index of Z, out and Psi fits
  const double lim = 4294967295.0;
  const bool i32 = static_cast<double>(n_in) * nd * Qin < lim && static_cast<double>(t1 - t0 + TS) * nd * Qin < lim &&
                   static_cast<double>(r1) * Qs < lim;
  ProfScope pr(K_COEF, 11 + 32 * prec_code<S>(), s,
               (static_cast<double>(n_in) * nd * Qin + rows * nd * Qin + static_cast<double>(R) * Qs) * sizeof(S), fl);
#define CF(P_, K_)                                                                                                \
  do {                                                                                                            \
    bool done_ = false;                                                                                           \
    if constexpr (f64) {                                                                                          \
      if (R <= 4) {                                                                                               \
        hipLaunchKernelGGL((k_coef_fused_pf<S, C, P_, K_, TS, 4, true>), g, dim3(TPB), 0, s, T, Psi, r0, R, Nt, t0, t1, Z, n_in, in_base, Bl, efirst, chunks, nd, Qin, out, Qs, nslab, ncb, nchunk); \
        done_ = true;                                                                                             \
      }                                                                                                           \
    }                                                                                                             \
    if (!done_ && R <= 4 && i32) hipLaunchKernelGGL((k_coef_fused<S, C, P_, K_, TS, 4, uint32_t>), g, dim3(TPB), 0, s, T, Psi, r0, R, Nt, t0, t1, Z, n_in, in_base, Bl, efirst, chunks, nd, Qin, out, Qs, nslab, ncb, nchunk); \
    else if (!done_ && R <= 4) hipLaunchKernelGGL((k_coef_fused<S, C, P_, K_, TS, 4, int64_t>), g, dim3(TPB), 0, s, T, Psi, r0, R, Nt, t0, t1, Z, n_in, in_base, Bl, efirst, chunks, nd, Qin, out, Qs, nslab, ncb, nchunk); \
    else if (!done_) hipLaunchKernelGGL((k_coef_fused<S, C, P_, K_, TS, 0, int64_t>), g, dim3(TPB), 0, s, T, Psi, r0, R, Nt, t0, t1, Z, n_in, in_base, Bl, efirst, chunks, nd, Qin, out, Qs, nslab, ncb, nchunk); \
  } while (0)
#define CFP(P_)                 \
  switch (ps) {                 \
    case 1: CF(P_, 2); break;   \
    case 2: CF(P_, 3); break;   \
    case 3: CF(P_, 4); break;   \
    default: CF(P_, 5); break;  \
  }
  switch (pt) {
    case 1: CFP(1); break;
    case 2: CFP(2); break;
    case 3: CFP(3); break;
    case 4: CFP(4); break;
    default: CFP(5); break;
  }
#undef CFP
#undef CF
  return true;
}

template <class S, class C>
void dense_mode(const C* Ap, int n, int npad, const S* x, S* y, int64_t outer, int64_t inner, hipStream_t s) {
  const int64_t ncols = outer * inner;
  if (ncols == 0) return;
  const unsigned grid = static_cast<unsigned>((ncols + 63) / 64);
  const int NT = npad / 16;
  const size_t abytes = static_cast<size_t>(npad) * lds_stride<C>(npad) * sizeof(C);
  // the matrix goes to LDS up to 96 KB (gfx950 allows 160 KB per workgroup)
  const bool lds = abytes <= 96 * 1024;
  ProfScope ps(K_DENSE, 4 + 32 * prec_code<S>(), s, 2.0 * ncols * n * sizeof(S), 2.0 * ncols * n * n);
  if (inner == 1 && NT <= 9) {
    // one wave per block; 4 column tiles (64 rows) unless the accumulators
    // (FP64 beyond 4 row tiles) or the staged rows would not fit
    const int ER = (std::is_same<C, double>::value && NT > 4) ? 2 : 4;
    const size_t xbytes = static_cast<size_t>(16 * ER) * n * sizeof(S);
    if (xbytes <= 64 * 1024) {
      const unsigned gridR = static_cast<unsigned>((outer + 16 * ER - 1) / (16 * ER));
#define DMR(nt, e) case nt: hipLaunchKernelGGL((k_dense_rows<S, C, nt, e>), dim3(gridR), dim3(64), xbytes, s, Ap, n, npad, x, y, outer); break;
      if constexpr (std::is_same<C, double>::value) {
        switch (NT) { DMR(1, 4) DMR(2, 4) DMR(3, 4) DMR(4, 4) DMR(5, 2) DMR(6, 2) DMR(7, 2) DMR(8, 2) DMR(9, 2) default: break; }
      } else {
        switch (NT) { DMR(1, 4) DMR(2, 4) DMR(3, 4) DMR(4, 4) DMR(5, 4) DMR(6, 4) DMR(7, 4) DMR(8, 4) DMR(9, 4) default: break; }
      }
#undef DMR
      return;
    }
  }
  // columns per lane: 4 while the accumulators fit (FP32 up to 9 row tiles,
  // FP64 up to 4), else 2; the E-wide loads need inner % E == 0 and aligned x, y
  const bool f64 = std::is_same<C, double>::value;
  const int ntmax4 = f64 ? 4 : 9;
  auto aligned = [&](int e) {
    return inner % e == 0 && inner >= 4 * e && reinterpret_cast<uintptr_t>(x) % (e * sizeof(S)) == 0 &&
           reinterpret_cast<uintptr_t>(y) % (e * sizeof(S)) == 0;
  };
  const int E = (NT <= ntmax4 && aligned(4)) ? 4 : (NT <= 9 && aligned(2)) ? 2 : 1;
  if (E > 1) {
    // persistent blocks (a few per CU, each staging the matrix once) when the
    // matrix is staged in LDS; one group per block otherwise
    const int64_t groupsE = (ncols + 64 * E - 1) / (64 * E);
    const unsigned gridE = static_cast<unsigned>(lds ? std::min<int64_t>(groupsE, 2048) : groupsE);
#define DME(nt, e)                                                                                              \
  case nt:                                                                                                      \
    if (lds) hipLaunchKernelGGL((k_dense_modeE<S, C, nt, e, true>), dim3(gridE), dim3(256), abytes, s, Ap, n, npad, x, y, inner, ncols); \
    else hipLaunchKernelGGL((k_dense_modeE<S, C, nt, e, false>), dim3(gridE), dim3(256), 0, s, Ap, n, npad, x, y, inner, ncols);  \
    break;
    if (E == 4) {
      if constexpr (std::is_same<C, double>::value) {
        switch (NT) { DME(1, 4) DME(2, 4) DME(3, 4) DME(4, 4) default: break; }
      } else {
        switch (NT) { DME(1, 4) DME(2, 4) DME(3, 4) DME(4, 4) DME(5, 4) DME(6, 4) DME(7, 4) DME(8, 4) DME(9, 4) default: break; }
      }
    } else {
      switch (NT) { DME(1, 2) DME(2, 2) DME(3, 2) DME(4, 2) DME(5, 2) DME(6, 2) DME(7, 2) DME(8, 2) DME(9, 2) default: break; }
    }
#undef DME
    return;
  }
  if (NT <= 9) {
    // any inner extent: tiles of 16 EU columns inside one outer index
    const int EU = (std::is_same<C, double>::value ? NT <= 4 : true) ? 4 : 2;
    const int64_t groups = (ncols + 64 * EU - 1) / (64 * EU);
    const unsigned gridU = static_cast<unsigned>(lds ? std::min<int64_t>(groups, 2048) : groups);
#define DMU(nt, e)                                                                                              \
  case nt:                                                                                                      \
    if (lds) hipLaunchKernelGGL((k_dense_modeU<S, C, nt, e, true>), dim3(gridU), dim3(256), abytes, s, Ap, n, npad, x, y, inner, ncols); \
    else hipLaunchKernelGGL((k_dense_modeU<S, C, nt, e, false>), dim3(gridU), dim3(256), 0, s, Ap, n, npad, x, y, inner, ncols);  \
    break;
    if (EU == 4) {
      if constexpr (std::is_same<C, double>::value) {
        switch (NT) { DMU(1, 4) DMU(2, 4) DMU(3, 4) DMU(4, 4) default: break; }
      } else {
        switch (NT) { DMU(1, 4) DMU(2, 4) DMU(3, 4) DMU(4, 4) DMU(5, 4) DMU(6, 4) DMU(7, 4) DMU(8, 4) DMU(9, 4) default: break; }
      }
    } else {
      switch (NT) { DMU(5, 2) DMU(6, 2) DMU(7, 2) DMU(8, 2) DMU(9, 2) default: break; }
    }
#undef DMU
    return;
  }
#define DM_CASE(nt)                                                                                          \
  case nt:                                                                                                   \
    if (lds) hipLaunchKernelGGL((k_dense_mode<S, C, nt, true>), dim3(grid), dim3(256), abytes, s, Ap, n, npad, x, y, inner, ncols); \
    else hipLaunchKernelGGL((k_dense_mode<S, C, nt, false>), dim3(grid), dim3(256), 0, s, Ap, n, npad, x, y, inner, ncols);  \
    break;
  switch (NT) {
    DM_CASE(1) DM_CASE(2) DM_CASE(3) DM_CASE(4) DM_CASE(5) DM_CASE(6) DM_CASE(7) DM_CASE(8) DM_CASE(9)
    default: break;
  }
#undef DM_CASE
}

bool dense_mode_b16(const bf16* Ab, int n, int npad, const bf16* x, bf16* y, int64_t outer, int64_t inner,
                    hipStream_t s) {
  const int64_t ncols = outer * inner;
  if (ncols == 0) return true;
  const int NT = npad / 16;
  if (NT < 1 || NT > 9 || npad % 16 != 0) return false;
  if (inner == 1) {
    constexpr int E = 4;
    const size_t xbytes = static_cast<size_t>(16 * E) * n * sizeof(bf16);
    if (xbytes > 64 * 1024) return false;
    ProfScope ps(K_DENSE, 4 + 32 * 2, s, 2.0 * ncols * n * sizeof(bf16), 2.0 * ncols * n * n);
    const unsigned grid = static_cast<unsigned>((outer + 16 * E - 1) / (16 * E));
#define DRB(nt) case nt: hipLaunchKernelGGL((k_dense_rows_b16<nt, E>), dim3(grid), dim3(64), xbytes, s, Ab, n, npad, x, y, outer); break;
    switch (NT) { DRB(1) DRB(2) DRB(3) DRB(4) DRB(5) DRB(6) DRB(7) DRB(8) DRB(9) default: break; }
#undef DRB
    return true;
  }
  auto aligned = [&](int e) {
    return inner % e == 0 && inner >= 4 * e && reinterpret_cast<uintptr_t>(x) % (e * sizeof(bf16)) == 0 &&
           reinterpret_cast<uintptr_t>(y) % (e * sizeof(bf16)) == 0;
  };
  const int E = aligned(4) ? 4 : (aligned(2) ? 2 : 0);
  if (E == 0) return false;
  const size_t abytes = static_cast<size_t>(npad) * lds_stride_b16(npad) * sizeof(bf16);
  const int64_t groups = (ncols + 64 * E - 1) / (64 * E);
  const unsigned grid = static_cast<unsigned>(std::min<int64_t>(groups, 2048));
  ProfScope ps(K_DENSE, 4 + 32 * 2, s, 2.0 * ncols * n * sizeof(bf16), 2.0 * ncols * n * n);
#define DEB(nt, e) case nt: hipLaunchKernelGGL((k_dense_modeE_b16<nt, e>), dim3(grid), dim3(256), abytes, s, Ab, n, npad, x, y, inner, ncols); break;
  if (E == 4) {
    switch (NT) { DEB(1, 4) DEB(2, 4) DEB(3, 4) DEB(4, 4) DEB(5, 4) DEB(6, 4) DEB(7, 4) DEB(8, 4) DEB(9, 4) default: break; }
  } else {
    switch (NT) { DEB(1, 2) DEB(2, 2) DEB(3, 2) DEB(4, 2) DEB(5, 2) DEB(6, 2) DEB(7, 2) DEB(8, 2) DEB(9, 2) default: break; }
  }
#undef DEB
  return true;
}

template <class S, class C>
void arrowhead(const S* r, S* y, const C* lam, const C* mu, int np, const C* l, C sigma, C Cm, int Nt,
               int64_t Ns, hipStream_t s) {
  ProfScope ps(K_ARROW, 5 + 32 * prec_code<S>(), s, 2.0 * Nt * Ns * sizeof(S));
  hipLaunchKernelGGL((k_arrowhead<S, C>), dim3(grid_for(Ns)), dim3(TPB), 0, s, r, y, lam, mu, l, sigma, Cm, Nt, np, Ns);
}

void kprof_enable(bool on) { prof().on = on; }
void kprof_suppress(bool on) { t_prof_suppress = on; }
bool kprof_enabled() { return prof().on; }
void kprof_gather_class(int cls) { t_gather_cls = cls; }

void kprof_read(int cls, double* ms, int64_t* launches, double* bytes, double* flops, int reset) {
  ProfState& p = prof();
  double tot = 0.0, by = 0.0, fl = 0.0;
  int64_t n = 0;
  for (auto& r : p.rec) {
    if (cls < 100 ? r.cls != cls : r.fn != cls - 100) continue;
    hipEventSynchronize(r.b);
    float t = 0.0f;
    if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) tot += t;
    by += r.bytes;
    fl += r.flops;
    ++n;
  }
  if (ms) *ms = tot;
  if (launches) *launches = n;
  if (bytes) *bytes = by;
  if (flops) *flops = fl;
  if (reset) {
    for (auto& r : p.rec) hipEventSynchronize(r.b);
    p.rec.clear();
    p.used = 0;
  }
}

bool kprof_record(int64_t i, int* fn, double* ms, double* bytes, double* flops) {
  ProfState& p = prof();
  if (i < 0 || i >= static_cast<int64_t>(p.rec.size())) return false;
  const auto& r = p.rec[static_cast<size_t>(i)];
  hipEventSynchronize(r.b);
  float t = 0.0f;
  hipEventElapsedTime(&t, r.a, r.b);
  if (fn) *fn = r.fn;
  if (ms) *ms = t;
  if (bytes) *bytes = r.bytes;
  if (flops) *flops = r.flops;
  return true;
}

template <class S>
bool time_core(const float* UtT, const float* Ut, int Nt, int npad, const S* x, S* z, int64_t Ns, const float* lam,
               const float* mu, int np, const float* l, float sigma, float Cm, hipStream_t s) {
  if (npad < 16 || npad > 64 || npad % 16 != 0 || Nt < 2 || Nt > npad || 2 * np > Nt - 1) return false;
  if (Ns <= 0) return true;
  const size_t lds = (2 * static_cast<size_t>(npad) * lds_stride<float>(npad) +
                      static_cast<size_t>(TC_WAVES) * npad * TC_W) * sizeof(float);
  // two blocks of TC_WAVES waves per CU (LDS bound) on 256 CUs
  const int64_t ntiles = (Ns + 15) / 16;
  const unsigned grid = static_cast<unsigned>(std::min<int64_t>((ntiles + TC_WAVES - 1) / TC_WAVES, 512));
  ProfScope ps(K_DENSE, 14 + 32 * prec_code<S>(), s, 2.0 * Nt * Ns * sizeof(S) + Ns * sizeof(float),
               4.0 * Nt * Nt * Ns + 12.0 * Nt * Ns);
#define TCK(nt) hipLaunchKernelGGL((k_time_core<S, nt>), dim3(grid), dim3(64 * TC_WAVES), lds, s, UtT, Ut, Nt, npad, x, z, Ns, lam, mu, np, l, sigma, Cm)
  switch (npad / 16) {
    case 1: TCK(1); break;
    case 2: TCK(2); break;
    case 3: TCK(3); break;
    default: TCK(4); break;
  }
#undef TCK
  return true;
}

int reduce_blocks(int64_t n) { return static_cast<int>((n + RED_CHUNK - 1) / RED_CHUNK); }

template <class T>
void multidot_partial(const T* V, int64_t ldv, int k, const T* w, int64_t n, double* part, int nb, hipStream_t s) {
  ProfScope ps(K_MULTIDOT, 6 + 32 * prec_code<T>(), s, (k + 1.0) * n * sizeof(T));
  constexpr int VEC = 16 / sizeof(T);
  if (ldv % VEC == 0 && reinterpret_cast<uintptr_t>(V) % 16 == 0 && reinterpret_cast<uintptr_t>(w) % 16 == 0)
    hipLaunchKernelGGL((k_multidot_v<T, VEC>), dim3(nb), dim3(TPB), 0, s, V, ldv, k, w, n, part);
  else
    hipLaunchKernelGGL((k_multidot<T>), dim3(nb), dim3(TPB), 0, s, V, ldv, k, w, n, part);
}
template <class T>
void multidot2_partial(const T* V, int64_t ldv, int k, const T* a, const T* b, int64_t n, double* part, int nb,
                       hipStream_t s) {
  ProfScope ps(K_MULTIDOT, 6 + 32 * prec_code<T>(), s, (k + 2.0) * n * sizeof(T));
  constexpr int VEC = 16 / sizeof(T);
  if (ldv % VEC == 0 && reinterpret_cast<uintptr_t>(V) % 16 == 0 && reinterpret_cast<uintptr_t>(a) % 16 == 0 &&
      reinterpret_cast<uintptr_t>(b) % 16 == 0)
    hipLaunchKernelGGL((k_multidot2<T, VEC>), dim3(nb), dim3(TPB), 0, s, V, ldv, k, a, b, n, part);
  else
    hipLaunchKernelGGL((k_multidot2<T, 1>), dim3(nb), dim3(TPB), 0, s, V, ldv, k, a, b, n, part);
}
template <class T>
void dcgs_update_partial(T* V, int64_t ldv, int j, const double* dots, int64_t n, double* part, int nb, double* sc,
                         hipStream_t s) {
  ProfScope ps(K_UPDATE, 7 + 32 * prec_code<T>(), s, (j + 4.0) * n * sizeof(T));
  hipLaunchKernelGGL((k_dcgs_update<T>), dim3(nb), dim3(TPB), 0, s, V, ldv, j, dots, n, part, sc);
}
void finalize_sum(const double* part, int nb, int k, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_sum, dim3(k), dim3(TPB), 0, s, part, nb, k, out);
}
void norm_givens(const double* part, int nb, double* D, double* G, const GivensLayout& L, int m, int j,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_norm_givens, dim3(1), dim3(TPB), 0, s, part, nb, D, G, L, m, j);
}
void givens_solve(const double* G, const GivensLayout& L, int m, int jn, int snap_j, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_givens_solve, dim3(1), dim3(64), 0, s, G, L, m, jn, snap_j, y);
}
template <class T>
void update_norm_partial(const T* V, int64_t ldv, int k, const double* h, T* w, int64_t n, double* part, int nb,
                         hipStream_t s) {
  ProfScope ps(K_UPDATE, 7 + 32 * prec_code<T>(), s, (k + 2.0) * n * sizeof(T));
  hipLaunchKernelGGL((k_update_norm<T>), dim3(nb), dim3(TPB), 0, s, V, ldv, k, h, w, n, part);
}
void absmax_partial(const double* x, int64_t n, double* part, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_absmax, dim3(nb), dim3(TPB), 0, s, x, n, part);
}
void sumsq_partial(const double* x, int64_t n, double* part, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_sumsq, dim3(nb), dim3(TPB), 0, s, x, n, part);
}
void finalize_max(const double* part, int nb, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_max, dim3(1), dim3(TPB), 0, s, part, nb, out);
}
void finalize_max2(const double* part, int64_t nb, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_max2, dim3(2), dim3(TPB), 0, s, part, nb, out);
}
template <class T>
void scale_by_dev(T* x, int64_t n, const double* nrm2, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL((k_scale_by_dev<T>), dim3(grid_for(n)), dim3(TPB), 0, s, x, n, nrm2);
}
void sc_scale(double* R, const double* fac, const double* maxes, double Cm, double invT, int64_t Qs, int64_t n,
              hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_sc_scale, dim3(grid_for(n)), dim3(TPB), 0, s, R, fac, maxes, Cm, invT, Qs, n);
}
template <class T>
void scale_to(const double* x, double a, T* y, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL((k_scale_to<T>), dim3(grid_for(n)), dim3(TPB), 0, s, x, a, y, n);
}
template <class T>
void sub_from(const double* b, const T* y, double* r, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL((k_sub_from<T>), dim3(grid_for(n)), dim3(TPB), 0, s, b, y, r, n);
}
void axpy(double a, const double* x, double* y, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(TPB), 0, s, a, x, 1.0, y, n);
}
void axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(TPB), 0, s, a, x, b, y, n);
}
template <class T>
void combine(const T* Z, int64_t ldz, int k, const double* c, double* x, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL((k_combine<T>), dim3(grid_for(n)), dim3(TPB), 0, s, Z, ldz, k, c, x, n);
}
template <class A, class B>
void convert(const A* x, B* y, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL((k_convert<A, B>), dim3(grid_for(n)), dim3(TPB), 0, s, x, y, n);
}
void fill(double* x, double v, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(TPB), 0, s, x, v, n);
}
void pointwise_ionic(const double* u, const double* ut, const double* lap, const double* w, const double* wt_time,
                     const double* wt_space, int64_t Qs, int nq_t, double Cm, double a, double c1, double c2,
                     double* g, double* absR, double* part, int nb, hipStream_t s, const Source& f, int q0, int Q1,
                     int Q2, double* Cq, double* Rq) {
  const int64_t total = Qs * nq_t;
  (void)nb;
  ProfScope ps(K_POINTWISE, 8, s, 6.0 * total * sizeof(double));
  hipLaunchKernelGGL(k_pointwise_ionic, dim3(grid_for(total)), dim3(TPB), 0, s, u, ut, lap, w, wt_time, wt_space, Qs,
                     total, Cm, a, c1, c2, g, absR, part, f, q0, Q1, Q2, Cq, Rq);
}
int64_t quad_fused(int d, int ps, int nqt, const double* A0, const double* A1, const double* A2, const double* UT,
                   const double* WW, int nd, int64_t Qin, int ne, const double* B0, const double* B2,
                   const int* efirst, const int* chunks, int nchunk, const double* wt, const double* win,
                   const double* wd, double sL,
                   double sM, double sF, double Cm, double a, double c1, double c2, double* G, double* M, int nel_d,
                   double* part, int64_t boff, hipStream_t s, int n2, int Q1, const double* e0x2,
                   const double* e2x2, const int* f2x, const Source& f, int q0, double* Cq, double* Rq,
                   int64_t Qs) {
  if (d < 2 || d > 3 || ps < 1 || ps > 4 || nqt < 1 || nqt > 6) return -1;
  const bool x2 = e0x2 != nullptr;
  if (x2 && (d != 3 || !e2x2 || !f2x || Q1 <= 0 || n2 <= 0 || Qin % Q1 != 0)) return -1;
  // column blocks padded to a multiple of 8 (the padding columns are invalid
  // and contribute zeros), see the block order in k_quad_fused
  const dim3 g(static_cast<unsigned>(((Qin + 63) / 64 + 7) / 8 * 8), static_cast<unsigned>(ne),
               static_cast<unsigned>(nchunk));
  const dim3 blk(static_cast<unsigned>(64 * nqt));
  const double rows = static_cast<double>(ne) * nqt;
  const double in_bytes = x2 ? rows * nd * static_cast<double>(n2) * Q1 * 4.0
                             : rows * nd * static_cast<double>(Qin) * (d == 3 ? 5.0 : 4.0);
  ProfScope pr(K_POINTWISE, 12, s,
               (in_bytes + rows * nd * Qin * (G ? 1.0 : 0.0) + (M ? static_cast<double>(ne) * nel_d * Qin : 0.0) +
                static_cast<double>(nel_d) * (ps + 1) * Qin) * sizeof(double));
#define QF(D_, K_)                                                                                                \
  do {                                                                                                            \
    if (x2)                                                                                                       \
      hipLaunchKernelGGL((k_quad_fused<D_, K_, true>), g, blk, 0, s, A0, A1, A2, UT, WW, nd, Qin, B0, B2, efirst, \
                         chunks, wt, win, wd, sL, sM, sF, Cm, a, c1, c2, G, M, nel_d, part, boff, n2, Q1, e0x2,   \
                         e2x2, f2x, f, q0, Cq, Rq, Qs);                                                          \
    else                                                                                                          \
      hipLaunchKernelGGL((k_quad_fused<D_, K_, false>), g, blk, 0, s, A0, A1, A2, UT, WW, nd, Qin, B0, B2,       \
                         efirst, chunks, wt, win, wd, sL, sM, sF, Cm, a, c1, c2, G, M, nel_d, part, boff, 0, 1,   \
                         nullptr, nullptr, nullptr, f, q0, Cq, Rq, Qs);                                          \
  } while (0)
#define QFK(D_)                         \
  switch (ps) {                         \
    case 1: QF(D_, 2); break;           \
    case 2: QF(D_, 3); break;           \
    case 3: QF(D_, 4); break;           \
    default: QF(D_, 5); break;          \
  }
  if (d == 3) {
    QFK(3);
  } else {
    QFK(2);
  }
#undef QFK
#undef QF
  return static_cast<int64_t>(g.x) * g.y * g.z;
}
void theta_finish(double* th, int64_t n, const double* maxes, double Cm, double invT, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_theta_finish, dim3(grid_for(n)), dim3(TPB), 0, s, th, n, maxes, Cm, invT);
}
void react_grid(const double* u, const double* w, double* c, int64_t n, double a, double c1, double c2, int newton,
                hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_react_grid, dim3(grid_for(n)), dim3(TPB), 0, s, u, w, c, n, a, c1, c2, newton);
}
void gram_partial(const double* C, int m, int64_t n, double* part, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_gram, dim3(nb), dim3(TPB), static_cast<size_t>(m) * GRAM_CH * sizeof(double), s, C, m, n, part);
}
void right_factor(const double* C, int m, int64_t n, const double* U, const double* inv_s, int R, double* V,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_right_factor, dim3(grid_for(n)), dim3(TPB), 0, s, C, m, n, U, inv_s, R, V);
}
void scale_rows(double* Psi, int R, int64_t Qs, const double* wq, hipStream_t s) {
  const int64_t total = static_cast<int64_t>(R) * Qs;
  if (total > 0) hipLaunchKernelGGL(k_scale_rows, dim3(grid_for(total)), dim3(TPB), 0, s, Psi, total, Qs, wq);
}
void transpose_nr(const double* V, int64_t N, int R, double* out, hipStream_t s) {
  if (N * R > 0) hipLaunchKernelGGL(k_transpose_nr, dim3(grid_for(N * R)), dim3(TPB), 0, s, V, N, R, out);
}
void add_unknowns(double* u_full, const double* delta, double alpha, int64_t n_unk, int64_t Ns, hipStream_t s) {
  hipLaunchKernelGGL(k_add_unknowns, dim3(grid_for(n_unk)), dim3(TPB), 0, s, u_full, delta, alpha, n_unk, Ns);
}

// explicit instantiations
template void gather<double, double, double>(const DTable<double>&, const double*, double*, int64_t, int64_t, int,
                                             int, double, double, hipStream_t);
template void gather<float, float, float>(const DTable<float>&, const float*, float*, int64_t, int64_t, int, int,
                                          float, float, hipStream_t);
template void gather<bf16, bf16, float>(const DTable<float>&, const bf16*, bf16*, int64_t, int64_t, int, int, float,
                                        float, hipStream_t);
template void gather_rows<double, double, double>(const DTable<double>&, int, int, const double*, double*, int64_t,
                                                  int64_t, int, int, double, double, hipStream_t);
template bool gather_dual<double, double>(const DTable<double>&, const DTable<double>&, const double*, const double*,
                                          double*, double*, int64_t, int64_t, int, int, double, double, hipStream_t);
template bool gather_dual<float, float>(const DTable<float>&, const DTable<float>&, const float*, const float*, float*,
                                        float*, int64_t, int64_t, int, int, float, float, hipStream_t);
template bool coef_fused<double, double>(const double*, const double*, int, int, int, int, int, int, int,
                                         const double*, int, int, const double*, const int*, const int*, int, int,
                                         int64_t, double*, int64_t, hipStream_t);
template bool coef_fused<float, float>(const float*, const float*, int, int, int, int, int, int, int, const float*, int,
                                       int, const float*, const int*, const int*, int, int, int64_t, float*, int64_t,
                                       hipStream_t);
template void react_point<double, double>(const double*, int, int, const DTable<double>&, const double*,
                                          const double*, const int*, const int*, const double*, const double*, int64_t,
                                          int, int, int, double*, double, hipStream_t);
template void react_point<float, float>(const float*, int, int, const DTable<float>&, const float*, const float*,
                                        const int*, const int*, const float*, const float*, int64_t, int, int, int,
                                        float*, float, hipStream_t);
template bool band_solve<double, double>(const double*, int, int64_t, int, const double*, double*, hipStream_t);
template bool band_solve<float, float>(const float*, int, int64_t, int, const float*, float*, hipStream_t);
template bool band_solve<bf16, float>(const float*, int, int64_t, int, const bf16*, bf16*, hipStream_t);
template void time_mix<double, double>(const double*, const double*, int, int, int, int, int, int, const double*,
                                       int, int, double*, int64_t, hipStream_t);
template void time_mix<float, float>(const float*, const float*, int, int, int, int, int, int, const float*, int, int,
                                     float*, int64_t, hipStream_t);
template void dense_mode<double, double>(const double*, int, int, const double*, double*, int64_t, int64_t,
                                         hipStream_t);
template void dense_mode<float, float>(const float*, int, int, const float*, float*, int64_t, int64_t, hipStream_t);
template void dense_mode<bf16, float>(const float*, int, int, const bf16*, bf16*, int64_t, int64_t, hipStream_t);
template void arrowhead<double, double>(const double*, double*, const double*, const double*, int,
                                        const double*, double, double, int, int64_t, hipStream_t);
template void arrowhead<float, float>(const float*, float*, const float*, const float*, int, const float*,
                                      float, float, int, int64_t, hipStream_t);
template void arrowhead<bf16, float>(const bf16*, bf16*, const float*, const float*, int, const float*, float,
                                     float, int, int64_t, hipStream_t);
template void convert<double, float>(const double*, float*, int64_t, hipStream_t);
template void multidot_partial<double>(const double*, int64_t, int, const double*, int64_t, double*, int, hipStream_t);
template void multidot_partial<float>(const float*, int64_t, int, const float*, int64_t, double*, int, hipStream_t);
template bool time_core<float>(const float*, const float*, int, int, const float*, float*, int64_t, const float*,
                               const float*, int, const float*, float, float, hipStream_t);
template bool time_core<bf16>(const float*, const float*, int, int, const bf16*, bf16*, int64_t, const float*,
                              const float*, int, const float*, float, float, hipStream_t);
template void multidot2_partial<double>(const double*, int64_t, int, const double*, const double*, int64_t, double*,
                                        int, hipStream_t);
template void multidot2_partial<float>(const float*, int64_t, int, const float*, const float*, int64_t, double*, int,
                                       hipStream_t);
template void dcgs_update_partial<double>(double*, int64_t, int, const double*, int64_t, double*, int, double*,
                                          hipStream_t);
template void dcgs_update_partial<float>(float*, int64_t, int, const double*, int64_t, double*, int, double*,
                                         hipStream_t);
template void update_norm_partial<double>(const double*, int64_t, int, const double*, double*, int64_t, double*, int,
                                          hipStream_t);
template void update_norm_partial<float>(const float*, int64_t, int, const double*, float*, int64_t, double*, int,
                                         hipStream_t);
template void scale_by_dev<double>(double*, int64_t, const double*, hipStream_t);
template void scale_by_dev<float>(float*, int64_t, const double*, hipStream_t);
template void scale_to<double>(const double*, double, double*, int64_t, hipStream_t);
template void scale_to<float>(const double*, double, float*, int64_t, hipStream_t);
template void sub_from<double>(const double*, const double*, double*, int64_t, hipStream_t);
template void sub_from<float>(const double*, const float*, double*, int64_t, hipStream_t);
template void combine<double>(const double*, int64_t, int, const double*, double*, int64_t, hipStream_t);
template void combine<float>(const float*, int64_t, int, const double*, double*, int64_t, hipStream_t);
template void convert<float, bf16>(const float*, bf16*, int64_t, hipStream_t);
template void convert<bf16, float>(const bf16*, float*, int64_t, hipStream_t);
template void convert<float, double>(const float*, double*, int64_t, hipStream_t);
template void convert<double, bf16>(const double*, bf16*, int64_t, hipStream_t);
template void convert<bf16, double>(const bf16*, double*, int64_t, hipStream_t);

// ---------------------------------------------------------------- allocation-free scratch
// Intermediate vectors of the allocation-free preconditioner entry point: one
// file-scope array per GPU, loaded with the code object and held until the
// process ends.  Host code never uses the array's name as an address: its
// per-device address is resolved once per device (with that device current)
// and kept in g_scratch_ptr.
__device__ __align__(256) double scratch[NOALLOC_BUFS * NOALLOC_MAX_UNKNOWNS];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

bool noalloc_scratch_init(int device, std::string& err) {
  if (device < 0 || device >= MAX_DEVICES) {
    err = "device index out of range";
    return false;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return true;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    return false;
  }
  g_scratch_ptr[device] = static_cast<double*>(p);
  return true;
}

double* noalloc_scratch(int device) {
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace stiga
