// Sparse operators of the pencil and the polynomial filter on the device.
//
// The paper accesses A, M and M^{-1} only through matrix-vector products
// (Sec. 6.1); most of the work of the eigensolver is here.  Every kernel
// is bound by HBM bandwidth: vectors are blocks [rows][w] with the w = 3b
// entries of a displacement node (components x columns) contiguous, so a
// gather of a neighbour row is one contiguous 3b-element segment, a
// lane handles one (row, entry) pair and the CSR indices and values of a
// row are loaded once per row group and broadcast.
//
// M^{-1} and K_p^{-1}: Chebyshev iteration preconditioned by the diagonal,
// on the element bounds [lo, hi] of spec(D^{-1} M), written on iterates:
//   y_1 = D^{-1} f / theta,
//   y_{j+1} = y_j + rho_j rho_{j-1} (y_j - y_{j-1}) + (2 rho_j / delta) D^{-1} (f - M y_j),
//   rho_0 = delta/theta, rho_j = 1 / (2 theta/delta - rho_{j-1}).
// The last step of the M solve is fused with the three-term Chebyshev
// filter update (W_{k+1} = a1 (B W_k - c W_k) + a2 W_{k-1}, Y += mu W_{k+1}).
// With mass passes (ApplyCfg::mixP) the M solve of an FP64 filter runs as
// FP32 passes of the same iteration joined by FP64 residual corrections
// (mass_solve_mixed); the update is then fused into the final FP64 sum.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "nm_internal.h"

namespace nm {
namespace {

__device__ __forceinline__ int64_t gtid() { return nm_xcd_block() * blockDim.x + threadIdx.x; }

// ---- vector access: V consecutive elements of a row as one 8/16-byte load
template <class T, int V>
struct Vx {
  T v[V];
};
template <class T, int V>
__device__ __forceinline__ Vx<T, V> ldv(const T* __restrict__ p) {
  Vx<T, V> r;
  if constexpr (V == 1) {
    r.v[0] = *p;
  } else if constexpr (std::is_same<T, double>::value && V == 2) {
    double2 q = *reinterpret_cast<const double2*>(p);
    r.v[0] = q.x; r.v[1] = q.y;
  } else if constexpr (std::is_same<T, float>::value && V == 2) {
    float2 q = *reinterpret_cast<const float2*>(p);
    r.v[0] = q.x; r.v[1] = q.y;
  } else if constexpr (std::is_same<T, double>::value) {
    static_assert(V == 4, "double rows are read 1, 2 or 4 at a time");
    double2 q = *reinterpret_cast<const double2*>(p), t = *reinterpret_cast<const double2*>(p + 2);
    r.v[0] = q.x; r.v[1] = q.y; r.v[2] = t.x; r.v[3] = t.y;
  } else {
    float4 q = *reinterpret_cast<const float4*>(p);
    r.v[0] = q.x; r.v[1] = q.y; r.v[2] = q.z; r.v[3] = q.w;
  }
  return r;
}
template <class T, int V>
__device__ __forceinline__ void stv(T* __restrict__ p, const Vx<T, V>& r) {
  if constexpr (V == 1) {
    *p = r.v[0];
  } else if constexpr (std::is_same<T, double>::value && V == 2) {
    *reinterpret_cast<double2*>(p) = make_double2(r.v[0], r.v[1]);
  } else if constexpr (std::is_same<T, float>::value && V == 2) {
    *reinterpret_cast<float2*>(p) = make_float2(r.v[0], r.v[1]);
  } else if constexpr (std::is_same<T, double>::value) {
    static_assert(V == 4, "double rows are written 1, 2 or 4 at a time");
    *reinterpret_cast<double2*>(p) = make_double2(r.v[0], r.v[1]);
    *reinterpret_cast<double2*>(p + 2) = make_double2(r.v[2], r.v[3]);
  } else {
    *reinterpret_cast<float4*>(p) = make_float4(r.v[0], r.v[1], r.v[2], r.v[3]);
  }
}

// streaming (nontemporal) variants for operands read or written once per
// step, so they do not displace the gathered rows from L2
template <class T, int V>
__device__ __forceinline__ Vx<T, V> ldv_nt(const T* __restrict__ p) {
  Vx<T, V> r;
#pragma unroll
  for (int i = 0; i < V; ++i) r.v[i] = __builtin_nontemporal_load(p + i);
  return r;
}
template <class T, int V>
__device__ __forceinline__ void stv_nt(T* __restrict__ p, const Vx<T, V>& r) {
#pragma unroll
  for (int i = 0; i < V; ++i) __builtin_nontemporal_store(r.v[i], p + i);
}

// LDS staging of the CSR entries of the rows a workgroup touches: the
// workgroup's lanes cover rows [r0, r1]; their column indices and values
// are loaded cooperatively (coalesced) into LDS, so that each lane can then
// issue all gathers of its row back to back instead of a dependent
// index-load -> gather chain per nonzero.
constexpr int STAGE_CAP = 2048;
template <class T, int NV>
struct Stage {
  int32_t kbeg;
  bool ok;
};
template <class T, int NV>
__device__ __forceinline__ Stage<T, NV> stage_rows(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                  const T* __restrict__ val, uint32_t rows, uint32_t wl,
                                                  int32_t* s_col, T* s_val) {
  const uint32_t g0 = (uint32_t)nm_xcd_block() * blockDim.x;
  const uint32_t r0 = min(g0 / wl, rows - 1);
  const uint32_t r1 = min((g0 + blockDim.x - 1) / wl, rows - 1);
  const int32_t kb = rp[r0], ke = rp[r1 + 1];
  Stage<T, NV> st{kb, (ke - kb) <= STAGE_CAP};
  if (st.ok) {
    for (int32_t i = threadIdx.x; i < ke - kb; i += blockDim.x) {
      s_col[i] = col[kb + i];
#pragma unroll
      for (int q = 0; q < NV; ++q) s_val[NV * i + q] = val[(size_t)NV * (kb + i) + q];
    }
  }
  __syncthreads();
  return st;
}

// sum_k val[k] X[col[k] * w + e .. e + V) over the row's entries, from LDS
// (or global memory when the rows did not fit): 8 gathers in flight per lane
// cl / vl point at the first staged entry (entry index `base`) or at the
// global arrays (base 0); entries are read at cl[k - base], so no pointer
// outside an allocation is ever formed.  Callers pass the LDS arrays and the
// global arrays in separate calls, so that after inlining the compiler knows
// each pointer's address space: LDS reads become ds_read (not flat loads,
// which would occupy the texture-address unit that the gathers saturate).
// X may hold a narrower type TX than the values and the sum (FP32 rows, FP64 values).
template <class T, int V, int U = 8, class TX = T>
__device__ __forceinline__ Vx<T, V> row_spmv(const int32_t* cl, const T* vl, int32_t base, int32_t k0, int32_t k1,
                                             const TX* __restrict__ X, uint32_t w, uint32_t e) {
  Vx<T, V> acc;
#pragma unroll
  for (int i = 0; i < V; ++i) acc.v[i] = T(0);
  for (int32_t k = k0; k < k1; k += U) {
    uint32_t c[U];
    T a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      // past the row end: re-read the first entry (always valid) with weight 0
      const bool in = k + u < k1;
      const int32_t kk = (in ? k + u : k0) - base;
      c[u] = (uint32_t)cl[kk];
      const T av = vl[kk];
      a[u] = in ? av : T(0);
    }
    Vx<TX, V> x[U];
    // c * w + e < rows * w < 2^32 for every block a launch accepts (check_block)
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = ldv<TX, V>(X + (size_t)(c[u] * w + e));
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int i = 0; i < V; ++i) acc.v[i] += a[u] * (T)x[u].v[i];
  }
  return acc;
}

// flat index of this lane in a launch covering rows * (w / V) lanes
__device__ __forceinline__ uint32_t lane_id() { return (uint32_t)nm_xcd_block() * blockDim.x + threadIdx.x; }

// sum over the row's 3x3 blocks of block . X[col] for the three output
// components: 3 gathered V-vectors per block (columns v..v+V of the three
// components of the neighbour), shared by the three outputs; cl / vl as in
// row_spmv (LDS or global arrays, entry k at k - base).  Per output the
// products are added block by block, d = 0, 1, 2 within a block.
template <class T, int V, int U = 2>
__device__ __forceinline__ void ag_row(const int32_t* cl, const T* vl, int32_t base, int32_t k0, int32_t k1,
                                       const T* __restrict__ X, uint32_t w, uint32_t b, uint32_t v,
                                       Vx<T, V> (&acc)[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int i = 0; i < V; ++i) acc[c].v[i] = T(0);
  for (int32_t k = k0; k < k1; k += U) {
    uint32_t cc[U];
    bool in[U];
    int32_t kk[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      in[u] = k + u < k1;
      kk[u] = (in[u] ? k + u : k0) - base;
      cc[u] = (uint32_t)cl[kk[u]];
    }
    Vx<T, V> x[U][3];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int d = 0; d < 3; ++d) x[u][d] = ldv<T, V>(X + (size_t)(cc[u] * w + d * b + v));
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const T av = vl[9 * (size_t)kk[u] + 3 * c + d];
          const T a = in[u] ? av : T(0);
#pragma unroll
          for (int i = 0; i < V; ++i) acc[c].v[i] += a * x[u][d].v[i];
        }
  }
}

// F = A_G X [+ E_G S] ; optionally Y1 = D^{-1} F / theta (first Chebyshev iterate).
// Lane (row, column group of V): all three components, so each neighbour
// row is gathered once per row (b / V lanes, 3 gathered V-vectors each).
template <class T, int V>
__global__ __launch_bounds__(256) void k_apply_ag(uint32_t N, uint32_t b, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col, const T* __restrict__ ag,
                                                  const T* __restrict__ X, const int32_t* __restrict__ egp,
                                                  const int32_t* __restrict__ egc, const T* __restrict__ egv,
                                                  const T* __restrict__ S, T* __restrict__ F,
                                                  const T* __restrict__ dinv, T inv_theta, T* __restrict__ Y1) {
  constexpr int CAP = STAGE_CAP / 4;
  constexpr int PV = 16 / sizeof(T);  // values per 16-byte piece
  __shared__ __align__(16) int32_t s_col[CAP + 4];
  __shared__ __align__(16) T s_val[9 * CAP + PV];
  const uint32_t w = 3 * b, bl = b / V;
  const uint32_t g = lane_id();
  const bool active = g < N * bl;
  // stage (indices and 3x3 blocks) of this workgroup's rows: whole 16-byte
  // pieces from the 16-byte boundary at or below the first entry, with
  // nontemporal loads (each block is read once per product, so it should not
  // displace gathered rows from L2), and the few entries past the last whole
  // piece one by one
  typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
  const uint32_t g0 = (uint32_t)nm_xcd_block() * blockDim.x;
  const uint32_t r0 = min(g0 / bl, N - 1), r1 = min((g0 + blockDim.x - 1) / bl, N - 1);
  const int32_t kb = rp[r0], ke = rp[r1 + 1];
  const bool staged = ke - kb <= CAP;
  const int32_t cb = kb & ~3;
  const int64_t vb = (9 * (int64_t)kb) & ~(int64_t)(PV - 1), ve = 9 * (int64_t)ke;
  if (staged) {
    const int32_t nc = (ke - cb) >> 2;
    const i32x4* sc = reinterpret_cast<const i32x4*>(col + cb);
    for (int32_t i = threadIdx.x; i < nc; i += blockDim.x)
      reinterpret_cast<i32x4*>(s_col)[i] = __builtin_nontemporal_load(sc + i);
    for (int32_t i = cb + 4 * nc + threadIdx.x; i < ke; i += blockDim.x) s_col[i - cb] = col[i];
    const int32_t nv = (int32_t)((ve - vb) / PV);
    const i32x4* sv = reinterpret_cast<const i32x4*>(ag + vb);
    for (int32_t i = threadIdx.x; i < nv; i += blockDim.x)
      reinterpret_cast<i32x4*>(s_val)[i] = __builtin_nontemporal_load(sv + i);
    for (int64_t i = vb + (int64_t)PV * nv + threadIdx.x; i < ve; i += blockDim.x) s_val[i - vb] = ag[i];
  }
  __syncthreads();
  if (!active) return;
  const uint32_t row = g / bl;
  const uint32_t v = (g - row * bl) * V;
  const int32_t k0 = rp[row], k1 = rp[row + 1];
  Vx<T, V> acc[3];
  if (staged)
    ag_row<T, V>(s_col + (kb - cb), s_val + (9 * (int64_t)kb - vb), kb, k0, k1, X, w, b, v, acc);
  else
    ag_row<T, V>(col, ag, 0, k0, k1, X, w, b, v, acc);
  if (S) {
    for (int32_t q = egp[row]; q < egp[row + 1]; ++q) {
      const Vx<T, V> sv = ldv<T, V>(S + (size_t)((uint32_t)egc[q] * b + v));
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T ev = egv[3 * (size_t)q + c];
#pragma unroll
        for (int i = 0; i < V; ++i) acc[c].v[i] += ev * sv.v[i];
      }
    }
  }
  const T sc = Y1 ? dinv[row] * inv_theta : T(0);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const size_t o = (size_t)row * w + c * b + v;
    if (F) stv<T, V>(F + o, acc[c]);
    if (Y1) {
      Vx<T, V> y;
#pragma unroll
      for (int i = 0; i < V; ++i) y.v[i] = sc * acc[c].v[i];
      stv<T, V>(Y1 + o, y);
    }
  }
}

// T_p = E_G^T X  (pressure rows, b entries)
template <class T>
__global__ __launch_bounds__(256) void k_egt(int64_t NP, int b, const int32_t* __restrict__ p,
                                             const int32_t* __restrict__ c, const T* __restrict__ val,
                                             const T* __restrict__ X, T* __restrict__ out) {
  int64_t g = gtid();
  if (g >= NP * b) return;
  int64_t row = g / b;
  int v = (int)(g - row * b);
  const int w = 3 * b;
  T acc = 0;
  for (int32_t k = p[row]; k < p[row + 1]; ++k) {
    const T* x = X + (int64_t)c[k] * w + v;
    const T* e = val + 3 * (int64_t)k;
    acc += e[0] * x[0] + e[1] * x[b] + e[2] * x[2 * b];
  }
  out[g] = acc;
}

// Y = E_G S (displacement rows)
template <class T>
__global__ __launch_bounds__(256) void k_eg(int64_t N, int b, const int32_t* __restrict__ p,
                                            const int32_t* __restrict__ c, const T* __restrict__ val,
                                            const T* __restrict__ S, T* __restrict__ Y) {
  const int w = 3 * b;
  int64_t g = gtid();
  if (g >= N * w) return;
  int64_t row = g / w;
  int e = (int)(g - row * w);
  int cc = e / b, v = e - cc * b;
  T acc = 0;
  for (int32_t k = p[row]; k < p[row + 1]; ++k) acc += val[3 * (int64_t)k + cc] * S[(int64_t)c[k] * b + v];
  Y[g] = acc;
}

// Y = (S (x) I_w) X for a scalar CSR S and row width w
template <class T, int V>
__global__ __launch_bounds__(256) void k_spmm_scalar(uint32_t rows, uint32_t w, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ col, const T* __restrict__ val,
                                                     const T* __restrict__ X, T* __restrict__ Y) {
  __shared__ int32_t s_col[STAGE_CAP];
  __shared__ T s_val[STAGE_CAP];
  const uint32_t wl = w / V;
  const uint32_t g = lane_id();
  auto sg = stage_rows<T, 1>(rp, col, val, rows, wl, s_col, s_val);
  if (g >= rows * wl) return;
  const uint32_t row = g / wl, e = (g - row * wl) * V;
  const int32_t k0 = rp[row], k1 = rp[row + 1];
  const Vx<T, V> acc = sg.ok ? row_spmv<T, V>(s_col, s_val, sg.kbeg, k0, k1, X, w, e)
                             : row_spmv<T, V>(col, val, 0, k0, k1, X, w, e);
  stv<T, V>(Y + (size_t)row * w + e, acc);
}

// Y = (M_s (x) [Omega]_x) X
template <class T>
__global__ __launch_bounds__(256) void k_spmm_coriolis(int64_t N, int b, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ col, const T* __restrict__ ms,
                                                       T o0, T o1, T o2, const T* __restrict__ X, T* __restrict__ Y) {
  const int w = 3 * b;
  int64_t g = gtid();
  if (g >= N * w) return;
  int64_t row = g / w;
  int e = (int)(g - row * w);
  int c = e / b, v = e - c * b;
  T s0 = 0, s1 = 0, s2 = 0;
  for (int32_t k = rp[row]; k < rp[row + 1]; ++k) {
    const T m = ms[k];
    const T* x = X + (int64_t)col[k] * w + v;
    s0 += m * x[0];
    s1 += m * x[b];
    s2 += m * x[2 * b];
  }
  // (Omega x s)_c
  T r = c == 0 ? (o1 * s2 - o2 * s1) : (c == 1 ? (o2 * s0 - o0 * s2) : (o0 * s1 - o1 * s0));
  Y[g] = r;
}

template <class T, int V>
__global__ __launch_bounds__(256) void k_cj_first(uint32_t rows, uint32_t w, const T* __restrict__ dinv,
                                                  const T* __restrict__ f, T inv_theta, T* __restrict__ y) {
  const uint32_t wl = w / V;
  const uint32_t g = lane_id();
  if (g >= rows * wl) return;
  const uint32_t row = g / wl, e = (g - row * wl) * V;
  const size_t o = (size_t)row * w + e;
  Vx<T, V> x = ldv<T, V>(f + o);
  const T sc = dinv[row] * inv_theta;
#pragma unroll
  for (int i = 0; i < V; ++i) x.v[i] *= sc;
  stv<T, V>(y + o, x);
}

// filter-series coefficients of the V entries starting at column j of a row
// [3][b]: one value for all columns, or per column (slices batched in one
// block, each with its own polynomial)
template <class T, int V>
__device__ __forceinline__ void series_coef(T mu0, T mu, const T* __restrict__ mu0c, const T* __restrict__ muc,
                                            uint32_t j, T (&m0)[V], T (&m1)[V]) {
#pragma unroll
  for (int i = 0; i < V; ++i) {
    m0[i] = muc ? (mu0c ? mu0c[j + i] : T(0)) : mu0;
    m1[i] = muc ? muc[j + i] : mu;
  }
}

// One Chebyshev-Jacobi step.  mode 0: out = y_{j+1}.  mode 1: filter update
// with z = y_{j+1}:  wout = a1 (z - cs win) + a2 wprev;
// ymode 1: Yacc = mu0 win + mu wout; ymode 2: Yacc += mu wout.
// out may alias yprev (same element read then written by one lane), wout
// may alias wprev.
template <class T, int V>
__global__ __launch_bounds__(256) void k_cj_step(uint32_t rows, uint32_t w, const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ col, const T* __restrict__ val,
                                                 const T* __restrict__ dinv, const T* __restrict__ f,
                                                 const T* __restrict__ ycur, const T* yprev, T alpha, T beta,
                                                 int prev_zero, int mode, T* out, const T* __restrict__ win,
                                                 const T* wprev, T a1, T cs, T a2, int ymode, T mu0, T mu,
                                                 const T* __restrict__ mu0c, const T* __restrict__ muc, T* wout,
                                                 T* Yacc) {
  __shared__ int32_t s_col[STAGE_CAP];
  __shared__ T s_val[STAGE_CAP];
  const uint32_t wl = w / V;
  const uint32_t g = lane_id();
  auto sg = stage_rows<T, 1>(rp, col, val, rows, wl, s_col, s_val);
  if (g >= rows * wl) return;
  const uint32_t row = g / wl, e = (g - row * wl) * V;
  const size_t o = (size_t)row * w + e;
  // own-row operands first, so their latency overlaps the gathers
  const Vx<T, V> yc = ldv<T, V>(ycur + o);
  const Vx<T, V> ff = ldv_nt<T, V>(f + o);
  Vx<T, V> yp;
  if (prev_zero) {
#pragma unroll
    for (int i = 0; i < V; ++i) yp.v[i] = T(0);
  } else {
    yp = ldv_nt<T, V>(yprev + o);
  }
  const T dr = dinv[row];
  const int32_t k0 = rp[row], k1 = rp[row + 1];
  const Vx<T, V> s = sg.ok ? row_spmv<T, V>(s_col, s_val, sg.kbeg, k0, k1, ycur, w, e)
                           : row_spmv<T, V>(col, val, 0, k0, k1, ycur, w, e);
  const T bd = beta * dr;
  Vx<T, V> z;
#pragma unroll
  for (int i = 0; i < V; ++i) z.v[i] = yc.v[i] + alpha * (yc.v[i] - yp.v[i]) + bd * (ff.v[i] - s.v[i]);
  if (mode == 0) {
    stv_nt<T, V>(out + o, z);
    return;
  }
  const Vx<T, V> wi = ldv<T, V>(win + o);
  Vx<T, V> wo;
#pragma unroll
  for (int i = 0; i < V; ++i) wo.v[i] = a1 * (z.v[i] - cs * wi.v[i]);
  if (a2 != T(0)) {
    const Vx<T, V> wp = ldv<T, V>(wprev + o);
#pragma unroll
    for (int i = 0; i < V; ++i) wo.v[i] += a2 * wp.v[i];
  }
  stv<T, V>(wout + o, wo);
  if (ymode == 0) return;
  T m0[V], m1[V];
  series_coef<T, V>(mu0, mu, mu0c, muc, e % (w / 3), m0, m1);
  if (ymode == 1) {
    Vx<T, V> yy;
#pragma unroll
    for (int i = 0; i < V; ++i) yy.v[i] = m0[i] * wi.v[i] + m1[i] * wo.v[i];
    stv<T, V>(Yacc + o, yy);
  } else if (ymode == 2) {
    Vx<T, V> yy = ldv<T, V>(Yacc + o);
#pragma unroll
    for (int i = 0; i < V; ++i) yy.v[i] += m1[i] * wo.v[i];
    stv<T, V>(Yacc + o, yy);
  }
}


// sum over the group's union columns of coef[., r] X[col] for the R rows;
// cl / cf as in row_spmv (LDS or global arrays): column entry l at
// cl[l - cbase], its R coefficients at cf[(l - fbase) R].  Entries past the
// group's end read entry l0 again (in range) with the coefficients scaled
// by 0, so every load is unconditional.
template <class T, int V, int R, int U = 4>
__device__ __forceinline__ void group_sum(const int32_t* cl, const T* cf, int32_t cbase, int32_t fbase, int32_t l0,
                                          int32_t l1, const T* __restrict__ X, uint32_t w, uint32_t e,
                                          Vx<T, V> (&acc)[R]) {
  for (int32_t l = l0; l < l1; l += U) {
    int32_t li[U];
    uint32_t c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      li[u] = l + u < l1 ? l + u : l0;
      c[u] = (uint32_t)cl[li[u] - cbase];
    }
    Vx<T, V> x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = ldv<T, V>(X + ((size_t)c[u] * w + e));
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const T* a = cf + (size_t)(li[u] - fbase) * R;
      T av[R];
#pragma unroll
      for (int r = 0; r < R; ++r) av[r] = a[r];
      const T keep = l + u < l1 ? T(1) : T(0);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const T ar = av[r] * keep;
#pragma unroll
        for (int i = 0; i < V; ++i) acc[r].v[i] += ar * x[u].v[i];
      }
    }
  }
}

// Row-group Chebyshev-Jacobi step (same arithmetic and modes as k_cj_step).
// Rows are processed in groups of R consecutive rows of the internal order;
// each lane owns one V-wide entry slot of all R rows and walks the union of
// their columns once, with an R-wide coefficient row per union column
// (zeros where a row lacks the column).  A gathered neighbour row serves
// every row of the group that touches it, so the number of gathers (which
// bound the step through the texture-address unit) drops by the ratio of
// the rows' entries to the size of their union.  Union columns and
// coefficients of the workgroup's groups are staged in LDS.
#define NM_CJ_GROUP_PARAMS                                                                                       \
  uint32_t N, uint32_t w, const int32_t *__restrict__ gptr, const int32_t *__restrict__ gcol,                      \
      const T *__restrict__ gcoef, const T *__restrict__ dinv, const T *__restrict__ f,                            \
      const T *__restrict__ ycur, const T *yprev, T alpha, T beta, int prev_zero, int mode, T *out,                \
      const T *__restrict__ win, const T *wprev, T a1, T cs, T a2, int ymode, T mu0, T mu,                         \
      const T *__restrict__ mu0c, const T *__restrict__ muc, T *wout, T *Yacc
#define NM_CJ_GROUP_ARGS                                                                                         \
  N, w, gptr, gcol, gcoef, dinv, f, ycur, yprev, alpha, beta, prev_zero, mode, out, win, wprev, a1, cs, a2, ymode, \
      mu0, mu, mu0c, muc, wout, Yacc
// one workgroup's share: the groups whose lanes fall in [vblock * 256, vblock * 256 + 256)
template <class T, int V, int R, int U, int GC>
__device__ __forceinline__ void cj_group_block(uint32_t vblock, NM_CJ_GROUP_PARAMS) {
  // LDS stage: 640 union entries in FP64 (23 KB), 896 in FP32 (18 KB, so 8
  // workgroups fit a CU; measured 3 % faster than 1280 at C2, 32 columns).
  // The waves-per-SIMD hint asks for at most 64 VGPRs, which the FP32 4-row
  // kernel at 16-byte rows meets without spilling (8 waves per SIMD, as
  // many as the LDS stage allows)
  constexpr int GCAP = GC > 0 ? GC : (sizeof(T) == 8 ? 640 : 896);
  static_assert(GCAP % 4 == 0 && (R * sizeof(T)) % 16 == 0, "16-byte LDS staging");
  __shared__ __align__(16) int32_t s_col[GCAP];
  __shared__ __align__(16) T s_cf[GCAP * R];
  __shared__ int32_t s_gp[256 + 2];  // union bounds of the workgroup's groups (at most 256 + 1 of them)
  const uint32_t wl = w / V;
  const uint32_t ngroups = (N + R - 1) / R;
  const uint32_t g0 = vblock * blockDim.x;
  const uint32_t g = g0 + threadIdx.x;
  const uint32_t G0 = min(g0 / wl, ngroups - 1), G1 = min((g0 + blockDim.x - 1) / wl, ngroups - 1);
  const int32_t lb = gptr[G0], le = gptr[G1 + 1];
  for (uint32_t i = threadIdx.x; i < G1 - G0 + 2; i += blockDim.x) s_gp[i] = gptr[G0 + i];
  // columns staged from lb rounded down to 4 entries (the union list is
  // padded by 4 entries at its end), coefficients from lb: both copied in
  // 16-byte pieces, with nontemporal loads (each entry is read by one
  // workgroup once per step, so it should not displace gathered rows from L2)
  typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
  const int32_t cb = lb & ~3;
  const bool staged = le - cb <= GCAP;
  if (staged) {
    const int32_t nc = (le - cb + 3) >> 2;
    const i32x4* sc = reinterpret_cast<const i32x4*>(gcol + cb);
    for (int32_t i = threadIdx.x; i < nc; i += blockDim.x)
      reinterpret_cast<i32x4*>(s_col)[i] = __builtin_nontemporal_load(sc + i);
    const int32_t nq = (int32_t)((size_t)(le - lb) * R * sizeof(T) / 16);
    const i32x4* sf = reinterpret_cast<const i32x4*>(gcoef + (size_t)lb * R);
    for (int32_t i = threadIdx.x; i < nq; i += blockDim.x)
      reinterpret_cast<i32x4*>(s_cf)[i] = __builtin_nontemporal_load(sf + i);
  }
  __syncthreads();
  if (g >= ngroups * wl) return;
  const uint32_t grp = g / wl, e = (g - grp * wl) * V;
  const uint32_t r0 = grp * R;
  Vx<T, V> acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int i = 0; i < V; ++i) acc[r].v[i] = T(0);
  const int32_t l0 = s_gp[grp - G0], l1 = s_gp[grp - G0 + 1];
  if (staged)
    group_sum<T, V, R, U>(s_col, s_cf, cb, lb, l0, l1, ycur, w, e, acc);
  else
    group_sum<T, V, R, U>(gcol, gcoef, 0, 0, l0, l1, ycur, w, e, acc);
  // the group's R diagonal entries in one piece (all R rows exist except in the last group)
  T dv[R];
  if (r0 + R <= N) {
#pragma unroll
    for (int r = 0; r < R; ++r) dv[r] = dinv[r0 + r];
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) dv[r] = r0 + r < N ? dinv[r0 + r] : T(0);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t row = r0 + r;
    if (row >= N) break;
    const size_t o = (size_t)row * w + e;
    const Vx<T, V> yc = ldv<T, V>(ycur + o);
    const Vx<T, V> ff = ldv_nt<T, V>(f + o);
    Vx<T, V> yp;
    if (prev_zero) {
#pragma unroll
      for (int i = 0; i < V; ++i) yp.v[i] = T(0);
    } else {
      yp = ldv_nt<T, V>(yprev + o);
    }
    const T bd = beta * dv[r];
    Vx<T, V> z;
#pragma unroll
    for (int i = 0; i < V; ++i) z.v[i] = yc.v[i] + alpha * (yc.v[i] - yp.v[i]) + bd * (ff.v[i] - acc[r].v[i]);
    if (mode == 0) {
      stv_nt<T, V>(out + o, z);
      continue;
    }
    const Vx<T, V> wi = ldv<T, V>(win + o);
    Vx<T, V> wo;
#pragma unroll
    for (int i = 0; i < V; ++i) wo.v[i] = a1 * (z.v[i] - cs * wi.v[i]);
    if (a2 != T(0)) {
      const Vx<T, V> wp = ldv<T, V>(wprev + o);
#pragma unroll
      for (int i = 0; i < V; ++i) wo.v[i] += a2 * wp.v[i];
    }
    stv<T, V>(wout + o, wo);
    if (ymode == 0) continue;
    T m0[V], m1[V];
    series_coef<T, V>(mu0, mu, mu0c, muc, e % (w / 3), m0, m1);
    if (ymode == 1) {
      Vx<T, V> yy;
#pragma unroll
      for (int i = 0; i < V; ++i) yy.v[i] = m0[i] * wi.v[i] + m1[i] * wo.v[i];
      stv<T, V>(Yacc + o, yy);
    } else if (ymode == 2) {
      Vx<T, V> yy = ldv<T, V>(Yacc + o);
#pragma unroll
      for (int i = 0; i < V; ++i) yy.v[i] += m1[i] * wo.v[i];
      stv<T, V>(Yacc + o, yy);
    }
  }
}


// one launch per step: workgroup i takes the i-th share of the XCD-aware order
template <class T, int V, int R, int U = 4, int GC = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_cj_group(NM_CJ_GROUP_PARAMS) {
  cj_group_block<T, V, R, U, GC>((uint32_t)nm_xcd_block(), NM_CJ_GROUP_ARGS);
}

// persistent form: as many workgroups as the GPU holds at once (a multiple
// of 8); the workgroups of XCD x sweep that XCD's contiguous eighth of the
// nvb shares in order, so the L2 of each XCD sees the same rows as in the
// one-share-per-workgroup launch, and every workgroup leaves its loop after
// at most ceil(nvb / gridDim.x) + 1 shares
template <class T, int V, int R, int U = 4, int GC = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_cj_group_persist(
    uint32_t nvb, NM_CJ_GROUP_PARAMS) {
  const uint32_t x = blockIdx.x & 7u, per = gridDim.x >> 3, k = blockIdx.x >> 3;
  const uint32_t span = (nvb + 7u) / 8u, lo = x * span, hi = min(nvb, lo + span);
  for (uint32_t vb = lo + k; vb < hi; vb += per) {
    cj_group_block<T, V, R, U, GC>(vb, NM_CJ_GROUP_ARGS);
    __syncthreads();  // the next share restages the LDS
  }
}
#undef NM_CJ_GROUP_PARAMS
#undef NM_CJ_GROUP_ARGS

// LDS-tiled Chebyshev-Jacobi step (same arithmetic, modes and summation
// order as k_cj_step, so the results are bit-identical).  A workgroup owns
// one tile of TR = 256 / LPR consecutive internal rows and one chunk of
// C = LPR * V consecutive entries of the row width w (V entries = 16 bytes
// per lane); each group of LPR lanes owns one row of the tile:
//   0. the own row's stream operands (f, y_prev, y, and the filter's) are
//      loaded first, so their latency overlaps the staging;
//   1. the chunk of every row in the tile's column union is gathered once
//      (LPR lanes per union row, 16-byte loads: first all union indices of
//      the lane, then all its chunks, all in flight together) and written to
//      LDS, next to the tile's CSR entries (16-bit union positions, values);
//   2. each row's sum runs from LDS in CSR order, then the update.
// A tile's union holds ~6.7 rows per row at TR = 32 against ~27.7 nonzeros
// per row, so neighbour chunks are read from L2 ~4x less often than by
// per-row gathers, as whole 64/128-byte segments.  Consecutive workgroups are
// the chunks of one tile (its entries stay in L2).  MAXJ and MAXE bound the
// union and the entries: U <= MAXJ * TR, E <= MAXE * 256 (launch plan).
template <class T, int LPR, int MAXJ, int MAXE>
__global__ __launch_bounds__(256) void k_cj_tile(
    uint32_t N, uint32_t w, int nch, int ucap, int ecap, const int32_t* __restrict__ tptr,
    const int32_t* __restrict__ tcol, const int32_t* __restrict__ rp, const uint16_t* __restrict__ lcol,
    const T* __restrict__ val, const T* __restrict__ dinv, const T* __restrict__ f, const T* __restrict__ ycur,
    const T* yprev, T alpha, T beta, int prev_zero, int mode, T* out, const T* __restrict__ win, const T* wprev, T a1,
    T cs, T a2, int ymode, T mu0, T mu, const T* __restrict__ mu0c, const T* __restrict__ muc, T* wout, T* Yacc) {
  constexpr int V = 16 / sizeof(T);
  constexpr int C = LPR * V;
  constexpr int TR = 256 / LPR;
  extern __shared__ float4 nm_tile_smem[];
  T* xs = reinterpret_cast<T*>(nm_tile_smem);                  // [ucap][C]
  T* s_val = xs + (size_t)ucap * C;                             // [ecap]
  uint16_t* s_lc = reinterpret_cast<uint16_t*>(s_val + ecap);  // [ecap]
  const uint32_t bid = (uint32_t)nm_xcd_block();
  const uint32_t tile = bid / (uint32_t)nch, ch = bid - tile * (uint32_t)nch;
  const uint32_t ntiles = (N + TR - 1) / TR;
  if (tile >= ntiles) return;  // grid padding: the whole workgroup leaves before any barrier
  const uint32_t r0 = tile * TR, r1 = min(N, r0 + (uint32_t)TR);
  const int32_t u0 = tptr[tile], U = tptr[tile + 1] - u0;
  const int32_t kb = rp[r0], E = rp[r1] - kb;
  const uint32_t lane = threadIdx.x % LPR, slot = threadIdx.x / LPR;
  const uint32_t e = ch * C + lane * V;  // entry of this lane within a row
  const uint32_t row = r0 + slot;
  const bool has = row < r1;
  const size_t o = (size_t)row * w + e;
  // 0. own-row operands (rows past the tile's end re-read its last row, a
  // valid address; loads are unconditional so no branch forces a wait)
  const uint32_t rowc = min(row, r1 - 1);
  const size_t oc = (size_t)rowc * w + e;
  const int32_t k0 = rp[rowc] - kb, k1 = rp[rowc + 1] - kb;
  const T dr = dinv[rowc];
  const Vx<T, V> ff = ldv_nt<T, V>(f + oc);
  const Vx<T, V> yp = ldv_nt<T, V>((prev_zero ? f : yprev) + oc);  // prev_zero: not used below
  const Vx<T, V> yc = ldv<T, V>(ycur + oc);
  Vx<T, V> wi, wp, yy;
  if (mode != 0) {  // uniform over the launch
    wi = ldv<T, V>(win + oc);
    wp = ldv<T, V>((a2 != T(0) ? wprev : win) + oc);
    yy = ldv<T, V>((ymode == 2 ? Yacc : win) + oc);
  }
  // 1. union indices, the tile's CSR entries (E <= MAXE * 256) and the union
  // chunks, all in flight before the LDS writes.  Loads are unconditional
  // (positions past the union or the entries re-read the last one, a valid
  // address) so that no branch forces a wait between them; only the LDS
  // writes are predicated.
  uint32_t ci[MAXJ];
#pragma unroll
  for (int j = 0; j < MAXJ; ++j) ci[j] = (uint32_t)tcol[u0 + min((int32_t)slot + j * TR, U - 1)];
  T vv[MAXE];
  uint16_t ll[MAXE];
#pragma unroll
  for (int q = 0; q < MAXE; ++q) {
    const int32_t i = min((int32_t)threadIdx.x + q * 256, E - 1);
    vv[q] = val[kb + i];
    ll[q] = lcol[kb + i];
  }
  Vx<T, V> xb[MAXJ];
#pragma unroll
  for (int j = 0; j < MAXJ; ++j) xb[j] = ldv<T, V>(ycur + (size_t)ci[j] * w + e);
#pragma unroll
  for (int q = 0; q < MAXE; ++q) {
    const int32_t i = (int32_t)threadIdx.x + q * 256;
    if (i < E) {
      s_val[i] = vv[q];
      s_lc[i] = ll[q];
    }
  }
#pragma unroll
  for (int j = 0; j < MAXJ; ++j) {
    const int32_t i = (int32_t)slot + j * TR;
    if (i < U) stv<T, V>(xs + (size_t)i * C + lane * V, xb[j]);
  }
  __syncthreads();
  if (!has) return;
  // 2. the row's sum from LDS in CSR order, then the update
  Vx<T, V> acc;
#pragma unroll
  for (int i = 0; i < V; ++i) acc.v[i] = T(0);
  int32_t k = k0;
  for (; k + 4 <= k1; k += 4) {
    T a[4];
    Vx<T, V> x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = s_val[k + u];
      x[u] = ldv<T, V>(xs + (size_t)s_lc[k + u] * C + lane * V);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int i = 0; i < V; ++i) acc.v[i] += a[u] * x[u].v[i];
  }
  for (; k < k1; ++k) {
    const T a = s_val[k];
    const Vx<T, V> x = ldv<T, V>(xs + (size_t)s_lc[k] * C + lane * V);
#pragma unroll
    for (int i = 0; i < V; ++i) acc.v[i] += a * x.v[i];
  }
  const T bd = beta * dr;
  Vx<T, V> z;
#pragma unroll
  for (int i = 0; i < V; ++i)
    z.v[i] = yc.v[i] + alpha * (yc.v[i] - (prev_zero ? T(0) : yp.v[i])) + bd * (ff.v[i] - acc.v[i]);
  if (mode == 0) {
    stv_nt<T, V>(out + o, z);
    return;
  }
  Vx<T, V> wo;
#pragma unroll
  for (int i = 0; i < V; ++i) wo.v[i] = a1 * (z.v[i] - cs * wi.v[i]);
  if (a2 != T(0)) {
#pragma unroll
    for (int i = 0; i < V; ++i) wo.v[i] += a2 * wp.v[i];
  }
  stv<T, V>(wout + o, wo);
  if (ymode == 0) return;
  T m0[V], m1[V];
  series_coef<T, V>(mu0, mu, mu0c, muc, e % (w / 3), m0, m1);
  if (ymode == 1) {
#pragma unroll
    for (int i = 0; i < V; ++i) yy.v[i] = m0[i] * wi.v[i] + m1[i] * wo.v[i];
    stv<T, V>(Yacc + o, yy);
  } else if (ymode == 2) {
#pragma unroll
    for (int i = 0; i < V; ++i) yy.v[i] += m1[i] * wo.v[i];
    stv<T, V>(Yacc + o, yy);
  }
}

// ---- mass solve in FP32 passes with FP64 residual corrections
// (iterative refinement of the Chebyshev-Jacobi solve): with r_0 = f, pass p
// solves M y_p = r_{p-1} in FP32 and r_p = r_{p-1} - M y_p is formed in FP64
// from the FP32 result (which converts to FP64 exactly, so r_p carries FP64
// rounding only); the solution y_1 + ... + y_P is summed in FP64.  With S the
// fixed-k solve the error operator is (I - S M)^P, so P passes of k steps
// reach the bound (2 r^k)^P of one FP64 pass of P k steps, while the rounding
// of each FP32 pass is relative to the correction it computes.

// pass 1, first iterate: f32 = f, y = D^{-1} f / theta (FP32)
template <int V>
__global__ __launch_bounds__(256) void k_mix_first(uint32_t rows, uint32_t w, const double* __restrict__ dinv,
                                                   const double* __restrict__ f, double inv_theta,
                                                   float* __restrict__ f32, float* __restrict__ y) {
  const uint32_t wl = w / V;
  const uint32_t g = lane_id();
  if (g >= rows * wl) return;
  const uint32_t row = g / wl, e = (g - row * wl) * V;
  const size_t o = (size_t)row * w + e;
  const Vx<double, V> x = ldv_nt<double, V>(f + o);
  const double sc = dinv[row] * inv_theta;
  Vx<float, V> a, b;
#pragma unroll
  for (int i = 0; i < V; ++i) {
    a.v[i] = (float)x.v[i];
    b.v[i] = (float)(sc * x.v[i]);
  }
  stv<float, V>(f32 + o, a);
  stv<float, V>(y + o, b);
}

// the FP64 sum of the passes so far plus this pass's y: acc_in (FP64) and
// y0 (the first pass's result, kept in FP32 until a second one is added)
// may each be absent
template <int V>
__device__ __forceinline__ Vx<double, V> pass_sum(const double* acc_in, const float* __restrict__ y0,
                                                  const Vx<float, V>& y, size_t o) {
  Vx<double, V> a;
  if (acc_in) {
    a = ldv<double, V>(acc_in + o);
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) a.v[i] = 0.0;
  }
  if (y0) {
    const Vx<float, V> q = ldv<float, V>(y0 + o);
#pragma unroll
    for (int i = 0; i < V; ++i) a.v[i] += (double)q.v[i];
  }
#pragma unroll
  for (int i = 0; i < V; ++i) a.v[i] += (double)y.v[i];
  return a;
}

// between passes: r = rin - M y (FP64, y the FP32 result of the pass),
// r32 = r, ynext = D^{-1} r / theta (first iterate of the next pass); rout
// (if set) = r for a later residual, acc_out (if set) = the sum of the
// passes so far (pass_sum).  rout may alias rin and acc_out acc_in (each lane
// reads, then writes, its own entries); y is only read.
template <int V>
__global__ __launch_bounds__(256) void k_mix_resid(uint32_t rows, uint32_t w, const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col, const double* __restrict__ val,
                                                   const double* __restrict__ dinv, const double* rin, double* rout,
                                                   const float* __restrict__ y, const double* acc_in,
                                                   const float* __restrict__ y0, double* acc_out, double inv_theta,
                                                   float* __restrict__ r32, float* __restrict__ ynext) {
  __shared__ int32_t s_col[STAGE_CAP];
  __shared__ double s_val[STAGE_CAP];
  const uint32_t wl = w / V;
  const uint32_t g = lane_id();
  auto sg = stage_rows<double, 1>(rp, col, val, rows, wl, s_col, s_val);
  if (g >= rows * wl) return;
  const uint32_t row = g / wl, e = (g - row * wl) * V;
  const size_t o = (size_t)row * w + e;
  const Vx<double, V> ri = ldv<double, V>(rin + o);
  const int32_t k0 = rp[row], k1 = rp[row + 1];
  const Vx<double, V> s = sg.ok ? row_spmv<double, V, 8, float>(s_col, s_val, sg.kbeg, k0, k1, y, w, e)
                                : row_spmv<double, V, 8, float>(col, val, 0, k0, k1, y, w, e);
  const double sc = dinv[row] * inv_theta;
  Vx<double, V> r;
  Vx<float, V> r3, yn;
#pragma unroll
  for (int i = 0; i < V; ++i) {
    r.v[i] = ri.v[i] - s.v[i];
    r3.v[i] = (float)r.v[i];
    yn.v[i] = (float)(sc * r.v[i]);
  }
  if (rout) stv<double, V>(rout + o, r);
  stv<float, V>(r32 + o, r3);
  stv<float, V>(ynext + o, yn);
  if (acc_out) stv<double, V>(acc_out + o, pass_sum<V>(acc_in, y0, ldv<float, V>(y + o), o));
}

// after the last pass: z = pass_sum (FP64), then as the last step of the
// FP64 solve: mode 0 out = z; mode 1 the filter update of k_cj_step
template <int V>
__global__ __launch_bounds__(256) void k_mix_final(uint32_t rows, uint32_t w, const double* __restrict__ acc_in,
                                                   const float* __restrict__ y0, const float* __restrict__ y,
                                                   int mode, double* out, const double* __restrict__ win,
                                                   const double* wprev, double a1, double cs, double a2, int ymode,
                                                   double mu0, double mu, const double* __restrict__ mu0c,
                                                   const double* __restrict__ muc, double* wout, double* Yacc) {
  const uint32_t wl = w / V;
  const uint32_t g = lane_id();
  if (g >= rows * wl) return;
  const uint32_t row = g / wl, e = (g - row * wl) * V;
  const size_t o = (size_t)row * w + e;
  const Vx<double, V> z = pass_sum<V>(acc_in, y0, ldv<float, V>(y + o), o);
  if (mode == 0) {
    stv<double, V>(out + o, z);
    return;
  }
  const Vx<double, V> wi = ldv<double, V>(win + o);
  Vx<double, V> wo;
#pragma unroll
  for (int i = 0; i < V; ++i) wo.v[i] = a1 * (z.v[i] - cs * wi.v[i]);
  if (a2 != 0.0) {
    const Vx<double, V> wp = ldv<double, V>(wprev + o);
#pragma unroll
    for (int i = 0; i < V; ++i) wo.v[i] += a2 * wp.v[i];
  }
  stv<double, V>(wout + o, wo);
  if (ymode == 0) return;
  double m0[V], m1[V];
  series_coef<double, V>(mu0, mu, mu0c, muc, e % (w / 3), m0, m1);
  if (ymode == 1) {
    Vx<double, V> yy;
#pragma unroll
    for (int i = 0; i < V; ++i) yy.v[i] = m0[i] * wi.v[i] + m1[i] * wo.v[i];
    stv<double, V>(Yacc + o, yy);
  } else if (ymode == 2) {
    Vx<double, V> yy = ldv<double, V>(Yacc + o);
#pragma unroll
    for (int i = 0; i < V; ++i) yy.v[i] += m1[i] * wo.v[i];
    stv<double, V>(Yacc + o, yy);
  }
}

template <class T>
__global__ void k_scale_copy(int64_t n, T a, const T* __restrict__ x, T* __restrict__ y) {
  int64_t g = gtid();
  if (g < n) y[g] = a * x[g];
}

__global__ void k_f64_f32(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  int64_t g = gtid();
  if (g < n) b[g] = (float)a[g];
}
__global__ void k_f32_f64(int64_t n, const float* __restrict__ a, double* __restrict__ b) {
  int64_t g = gtid();
  if (g < n) b[g] = (double)a[g];
}

// column dot products, stage 1: partial sums per workgroup (fixed order)
__global__ __launch_bounds__(256) void k_coldot_partial(int64_t rows, int nc, const double* __restrict__ X, int ldx,
                                                        const double* __restrict__ Y, int ldy, int64_t rows_per,
                                                        double* __restrict__ part) {
  // workgroup blockIdx.x handles rows [blk*rows_per, ...) for all nc columns
  __shared__ double red[256];
  int64_t r0 = (int64_t)blockIdx.x * rows_per, r1 = r0 + rows_per;
  if (r1 > rows) r1 = rows;
  for (int v = 0; v < nc; ++v) {
    double s = 0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) s += X[r * ldx + v] * Y[r * ldy + v];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * nc + v] = red[0];
    __syncthreads();
  }
}
__global__ void k_coldot_final(int nblk, int nc, const double* __restrict__ part, double* __restrict__ out) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nc) return;
  double s = 0;
  for (int i = 0; i < nblk; ++i) s += part[(int64_t)i * nc + v];
  out[v] = s;
}

// ---- launch helpers: V = elements per lane (16-byte loads where the row
// width allows), lanes = rows * (w / V)
template <class T>
int pick_v(uint32_t w) {
  if (std::is_same<T, float>::value && w % 4 == 0) return 4;
  return w % 2 == 0 ? 2 : 1;
}
#define NM_LAUNCH_V(KERN, T, V, lanes, st, ...)                                                         \
  do {                                                                                                 \
    if ((V) == 4)                                                                                      \
      hipLaunchKernelGGL((KERN<T, 4>), dim3(grid_for(lanes)), dim3(256), 0, st, __VA_ARGS__);           \
    else if ((V) == 2)                                                                                 \
      hipLaunchKernelGGL((KERN<T, 2>), dim3(grid_for(lanes)), dim3(256), 0, st, __VA_ARGS__);           \
    else                                                                                               \
      hipLaunchKernelGGL((KERN<T, 1>), dim3(grid_for(lanes)), dim3(256), 0, st, __VA_ARGS__);           \
  } while (0)

template <class T>
void launch_spmm_scalar(int64_t rows, int w, const int32_t* rp, const int32_t* col, const T* val, const T* X, T* Y,
                        hipStream_t st) {
  int v = pick_v<T>(w);
  NM_LAUNCH_V(k_spmm_scalar, T, v, rows * (w / v), st, (uint32_t)rows, (uint32_t)w, rp, col, val, X, Y);
}
template <class T>
void launch_cj_first(int64_t rows, int w, const T* dinv, const T* f, T inv_theta, T* y, hipStream_t st) {
  int v = pick_v<T>(w);
  NM_LAUNCH_V(k_cj_first, T, v, rows * (w / v), st, (uint32_t)rows, (uint32_t)w, dinv, f, inv_theta, y);
}
// row-group launch plan for the mass solve (displacement rows)
struct GroupPlan {
  bool on = false;
  bool persist = false;  // one persistent launch per step (k_cj_group_persist)
  int R = 0;
  const int32_t *gptr = nullptr, *gcol = nullptr;
  const void* gcoef = nullptr;
};
// By default only for blocks of at least 32 columns: narrower rows put more
// groups in a workgroup than its LDS stage holds (640 union entries in FP64,
// 896 in FP32).  FP32 at 32 columns on the 384k-tet planet: 0.343 vs
// 0.422 ms (grouped vs per-row).  grouped == 2 forces the grouped kernel at
// any width.
template <class T>
GroupPlan group_plan(const nm_pencil* P, int b) {
  GroupPlan tp;
  if (!P->grouped || P->grp_rows <= 0 || b < 1) return tp;
  if (P->grouped == 1 && b < 32) return tp;
  const void* cf = sizeof(T) == 8 ? (const void*)P->grp_coef.p : (const void*)P->grp_coef32.p;
  if (!cf) return tp;
  tp.on = true;
  tp.persist = P->persist > 0;
  tp.R = P->grp_rows;
  tp.gptr = P->grp_ptr.p;
  tp.gcol = P->grp_col.p;
  tp.gcoef = cf;
  return tp;
}

// LDS-tile launch plan: tiles of 32 rows read rows in 128-byte chunks (8
// lanes per row), tiles of 64 rows in 64-byte chunks (4 lanes); the chunk
// must divide the row, the largest union must fit MAXJ chunks per row slot
// and the workgroup's LDS (the largest union's chunks and the largest
// tile's CSR entries) must stay within 64 KB.
constexpr int TILE_MAXJ = 16;
struct TilePlan {
  bool on = false;
  int TR = 0, lpr = 0, nch = 0, ucap = 0, ecap = 0;
  size_t lds = 0;
};
template <class T>
TilePlan tile_plan(const nm_pencil* P, int b) {
  TilePlan t;
  if (!P->tiled || b < 1 || (P->tile_rows != 32 && P->tile_rows != 64)) return t;
  const size_t rowb = (size_t)3 * b * sizeof(T);
  const int lpr = 256 / P->tile_rows;
  const size_t chunk = (size_t)lpr * 16;
  if (rowb % chunk != 0) return t;
  if (P->tile_umax > TILE_MAXJ * P->tile_rows) return t;
  if (P->tile_emax > (P->tile_rows == 32 ? 8 : 12) * 256) return t;
  t.ucap = P->tile_umax;
  t.ecap = (P->tile_emax + 7) / 8 * 8;
  t.lds = t.ucap * chunk + (size_t)t.ecap * (sizeof(T) + 2);
  if (t.lds > 65536) return t;
  t.on = true;
  t.TR = P->tile_rows;
  t.lpr = lpr;
  t.nch = (int)(rowb / chunk);
  return t;
}

template <class T>
void launch_cj_tile(const nm_pencil* P, const TilePlan& tp, const T* val, int64_t N, int w, const T* dinv,
                    const T* f, const T* ycur, const T* yprev, T alpha, T beta, int prev_zero, int mode, T* out,
                    const T* win, const T* wprev, T a1, T cs, T a2, int ymode, T mu0, T mu, const T* mu0c,
                    const T* muc, T* wout, T* Yacc, hipStream_t st) {
  const int64_t ntiles = (N + tp.TR - 1) / tp.TR;
  const int64_t wgs = ntiles * tp.nch;
  unsigned g = (unsigned)((wgs + 7) / 8 * 8);
#define NM_TILE(LPR, MJ, ME)                                                                                      \
  hipLaunchKernelGGL((k_cj_tile<T, LPR, MJ, ME>), dim3(g), dim3(256), tp.lds, st, (uint32_t)N, (uint32_t)w, tp.nch, \
                     tp.ucap, tp.ecap, P->tile_ptr.p, P->tile_col.p, P->row_ptr.p, P->tile_lcol.p, val, dinv, f,   \
                     ycur, yprev, alpha, beta, prev_zero, mode, out, win, wprev, a1, cs, a2, ymode, mu0, mu, mu0c, \
                     muc, wout, Yacc)
  const int mj = (tp.ucap + tp.TR - 1) / tp.TR, me = (tp.ecap + 255) / 256;
  if (tp.lpr == 8) {
    if (mj <= 8) {
      if (me <= 4) NM_TILE(8, 8, 4); else NM_TILE(8, 8, 8);
    } else {
      if (me <= 4) NM_TILE(8, 16, 4); else NM_TILE(8, 16, 8);
    }
  } else {
    if (mj <= 8) {
      if (me <= 8) NM_TILE(4, 8, 8); else NM_TILE(4, 8, 12);
    } else {
      if (me <= 8) NM_TILE(4, 16, 8); else NM_TILE(4, 16, 12);
    }
  }
#undef NM_TILE
}

// workgroups of a persistent launch: the device's CUs times the workgroups
// of this kernel one CU holds, rounded down to a multiple of 8 (queried once
// per kernel and device)
template <class K>
unsigned persistent_grid(K kernel) {
  static std::mutex mx;
  static std::map<std::pair<const void*, int>, unsigned> cache;
  int dev = 0;
  NM_HIP(hipGetDevice(&dev));
  const std::pair<const void*, int> key((const void*)kernel, dev);
  std::lock_guard<std::mutex> lk(mx);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  NM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0));
  NM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const unsigned g = std::max(8u, (unsigned)(std::max(per_cu, 1) * std::max(cus, 1)) / 8u * 8u);
  cache[key] = g;
  return g;
}

template <class T>
void launch_cj_group(const GroupPlan& tp, int64_t N, int w, const T* dinv, const T* f, const T* ycur, const T* yprev,
                     T alpha, T beta, int prev_zero, int mode, T* out, const T* win, const T* wprev, T a1, T cs, T a2,
                     int ymode, T mu0, T mu, const T* mu0c, const T* muc, T* wout, T* Yacc, hipStream_t st) {
  const int v = pick_v<T>(w);
  const int64_t lanes = (N + tp.R - 1) / tp.R * (w / v);
  const uint32_t nvb = (uint32_t)((lanes + 255) / 256);
  const T* cf = (const T*)tp.gcoef;
#define NM_GRP(VV, RR)                                                                                               \
  do {                                                                                                               \
    if (tp.persist) {                                                                                                \
      const unsigned pg = persistent_grid(k_cj_group_persist<T, VV, RR>);                                            \
      hipLaunchKernelGGL((k_cj_group_persist<T, VV, RR>), dim3(std::min(pg, (nvb + 7u) / 8u * 8u)), dim3(256), 0, st, \
                         nvb, (uint32_t)N, (uint32_t)w, tp.gptr, tp.gcol, cf, dinv, f, ycur, yprev, alpha, beta,     \
                         prev_zero, mode, out, win, wprev, a1, cs, a2, ymode, mu0, mu, mu0c, muc, wout, Yacc);        \
    } else {                                                                                                         \
      hipLaunchKernelGGL((k_cj_group<T, VV, RR>), dim3(grid_for(lanes)), dim3(256), 0, st, (uint32_t)N, (uint32_t)w,  \
                         tp.gptr, tp.gcol, cf, dinv, f, ycur, yprev, alpha, beta, prev_zero, mode, out, win, wprev,  \
                         a1, cs, a2, ymode, mu0, mu, mu0c, muc, wout, Yacc);                                         \
    }                                                                                                                \
  } while (0)
  if (tp.R == 8) {
    if (v == 4) NM_GRP(4, 8); else if (v == 2) NM_GRP(2, 8); else NM_GRP(1, 8);
  } else {
    if (v == 4) NM_GRP(4, 4); else if (v == 2) NM_GRP(2, 4); else NM_GRP(1, 4);
  }
#undef NM_GRP
}

// Chebyshev-Jacobi step of the displacement mass solve: LDS tiles where
// they apply, else row groups, else one row per lane.  Pressure (K_p)
// solves pass no plans and take the per-row kernel.
template <class T>
struct MassPlan {
  const nm_pencil* P = nullptr;
  TilePlan tile;
  GroupPlan group;
};
template <class T>
MassPlan<T> mass_plan(const nm_pencil* P, int b) {
  MassPlan<T> m;
  m.P = P;
  m.tile = tile_plan<T>(P, b);
  if (!m.tile.on) m.group = group_plan<T>(P, b);
  return m;
}

template <class T>
void launch_cj_step(int64_t rows, int w, const int32_t* rp, const int32_t* col, const T* val, const T* dinv,
                    const T* f, const T* ycur, const T* yprev, T alpha, T beta, int prev_zero, int mode, T* out,
                    const T* win, const T* wprev, T a1, T cs, T a2, int ymode, T mu0, T mu, T* wout, T* Yacc,
                    hipStream_t st, const MassPlan<T>* mp = nullptr, const T* mu0c = nullptr,
                    const T* muc = nullptr) {
  if (mp && mp->tile.on) {
    launch_cj_tile<T>(mp->P, mp->tile, val, rows, w, dinv, f, ycur, yprev, alpha, beta, prev_zero, mode, out, win,
                      wprev, a1, cs, a2, ymode, mu0, mu, mu0c, muc, wout, Yacc, st);
    return;
  }
  const GroupPlan* tp = mp ? &mp->group : nullptr;
  if (tp && tp->on) {
    launch_cj_group<T>(*tp, rows, w, dinv, f, ycur, yprev, alpha, beta, prev_zero, mode, out, win, wprev, a1, cs,
                       a2, ymode, mu0, mu, mu0c, muc, wout, Yacc, st);
    return;
  }
  int v = pick_v<T>(w);
  NM_LAUNCH_V(k_cj_step, T, v, rows * (w / v), st, (uint32_t)rows, (uint32_t)w, rp, col, val, dinv, f, ycur, yprev,
              alpha, beta, prev_zero, mode, out, win, wprev, a1, cs, a2, ymode, mu0, mu, mu0c, muc, wout, Yacc);
}
template <class T>
void launch_apply_ag(int64_t N, int b, const int32_t* rp, const int32_t* col, const T* ag, const T* X,
                     const int32_t* egp, const int32_t* egc, const T* egv, const T* S, T* F, const T* dinv,
                     T inv_theta, T* Y1, hipStream_t st) {
  // two entries per lane (8- or 16-byte gathers): b / 2 lanes per row keeps a
  // workgroup's rows within the LDS stage at 32 columns
  const int v = b % 2 == 0 ? 2 : 1;
  NM_LAUNCH_V(k_apply_ag, T, v, N * (b / v), st, (uint32_t)N, (uint32_t)b, rp, col, ag, X, egp, egc, egv, S, F,
              dinv, inv_theta, Y1);
}

struct ChebCoef {
  double theta, delta, sigma;
  std::vector<double> alpha, beta;  // step j = 1..k-1
};
ChebCoef cheb_coef(double lo, double hi, int k) {
  ChebCoef c;
  c.theta = 0.5 * (hi + lo);
  c.delta = 0.5 * (hi - lo);
  c.sigma = c.theta / c.delta;
  double rho_prev = 1.0 / c.sigma;
  for (int j = 1; j < k; ++j) {
    double rho = 1.0 / (2.0 * c.sigma - rho_prev);
    c.alpha.push_back(rho * rho_prev);
    c.beta.push_back(2.0 * rho / c.delta);
    rho_prev = rho;
  }
  return c;
}

template <class T>
struct Mats {
  const T *ag, *ms, *mdinv, *kp, *kpdinv, *eg, *egt;
};
template <class T>
Mats<T> mats(const nm_pencil* P);
template <>
Mats<double> mats<double>(const nm_pencil* P) {
  return {P->ag.p, P->ms.p, P->mdinv.p, P->kp.p, P->kpdinv.p, P->eg_val.p, P->egt_val.p};
}
template <>
Mats<float> mats<float>(const nm_pencil* P) {
  return {P->ag32.p, P->ms32.p, P->mdinv32.p, P->kp32.p, P->kpdinv32.p, P->eg_val32.p, P->egt_val32.p};
}

#define LAUNCH(kern, threads, st, ...) \
  hipLaunchKernelGGL(kern, dim3(grid_for(threads)), dim3(256), 0, st, __VA_ARGS__)

// S_p(t): fixed-k Chebyshev-Jacobi solve with K_p; result pointer returned
template <class T>
T* kp_solve(const nm_pencil* P, int b, const T* t, int kP, T* pa, T* pb, hipStream_t st) {
  auto m = mats<T>(P);
  const int64_t NP = P->n_pres;
  ChebCoef cc = cheb_coef(P->ref.p_lo, P->ref.p_hi, kP);
  launch_cj_first<T>(NP, b, m.kpdinv, t, (T)(1.0 / cc.theta), pa, st);
  T *cur = pa, *prev = pb;
  for (int j = 1; j < kP; ++j) {
    launch_cj_step<T>(NP, b, P->kp_ptr.p, P->kp_col.p, m.kp, m.kpdinv, t, cur, prev, (T)cc.alpha[j - 1],
                      (T)cc.beta[j - 1], j == 1 ? 1 : 0, 0, prev, nullptr, nullptr, T(0), T(0), T(0), 0, T(0), T(0),
                      nullptr, nullptr, st);
    std::swap(cur, prev);
  }
  return cur;
}

// F = A X (Cowling operator) and optionally Y1 = D^{-1} F / theta
template <class T>
void a_apply(const nm_pencil* P, int b, const T* X, T* F, T* Y1, double inv_theta, int kP, const BWork<T>& w,
             hipStream_t st) {
  auto m = mats<T>(P);
  const T* S = nullptr;
  if (P->n_pres > 0) {
    LAUNCH(k_egt<T>, P->n_pres * b, st, P->n_pres, b, P->egt_ptr.p, P->egt_col.p, m.egt, X, w.pt);
    S = kp_solve<T>(P, b, w.pt, kP, w.pa, w.pb, st);
  }
  if constexpr (std::is_same<T, double>::value) {
    if (P->selfgrav) {
      // A X with the self-gravitation term -C^T S C X, then the first mass-solve iterate
      launch_apply_ag<T>(P->N, b, P->row_ptr.p, P->col.p, m.ag, X, P->eg_ptr.p, P->eg_col.p, m.eg, S, F, m.mdinv,
                         T(0), nullptr, st);
      selfgrav_add(P->selfgrav, b, X, F, st);
      if (Y1) launch_cj_first<T>(P->N, 3 * b, m.mdinv, F, (T)inv_theta, Y1, st);
      return;
    }
  } else {
    NM_REQUIRE(!P->selfgrav, NM_EINVAL, "self-gravitation runs with FP64 operators only");
  }
  launch_apply_ag<T>(P->N, b, P->row_ptr.p, P->col.p, m.ag, X, P->eg_ptr.p, P->eg_col.p, m.eg, S, F, m.mdinv,
                     (T)inv_theta, Y1, st);
}

struct Update {
  bool on = false;
  const void* win = nullptr;
  const void* wprev = nullptr;
  double a1 = 0, cs = 0, a2 = 0, mu0 = 0, mu = 0;
  int ymode = 0;
  void* wout = nullptr;
  void* Y = nullptr;
  const void* mu0c = nullptr;  // per-column series coefficients (device, or null: mu0 / mu)
  const void* muc = nullptr;
};

// work vectors of the mixed-precision mass solve, each [N][3b]
struct MixBufs {
  double *r64, *acc;  // FP64 residual, FP64 sum of the passes
  float* s[4];        // FP32 right-hand side, two iterates, first pass's result
};

// Mixed-precision mass solve: Z = S(f) (mode 0) or the filter update u with
// z = S(f), by cfg.mixP FP32 passes of cfg.mixK Chebyshev-Jacobi steps (see
// k_mix_first).
void mass_solve_mixed(const nm_pencil* P, int b, const double* f, double* Z, const Update& u, const ApplyCfg& cfg,
                      const MixBufs& w, hipStream_t st, KernelProf* prof) {
  NM_REQUIRE(cfg.mixP >= 2 && cfg.mixK >= 2, NM_EINVAL, "mixed mass solve needs >= 2 passes of >= 2 steps");
  NM_REQUIRE(P->ms32.p && P->mdinv32.p, NM_EINVAL, "mixed mass solve without the FP32 matrix shadows");
  const auto m64 = mats<double>(P);
  const auto m32 = mats<float>(P);
  const MassPlan<float> tp = mass_plan<float>(P, b);
  const ChebCoef cc = cheb_coef(P->ref.m_lo, P->ref.m_hi, cfg.mixK);
  const int64_t N = P->N;
  const int wd = 3 * b;
  const int v = wd % 4 == 0 ? 4 : (wd % 2 == 0 ? 2 : 1);
  const int64_t lanes = N * (wd / v);
  const double it = 1.0 / cc.theta;
  // FP32 buffers: right-hand side, two iterates, and the first pass's result
  // (kept in FP32 until the second pass's is added to it in FP64)
  float *rhs = w.s[0], *cur = w.s[1], *prev = w.s[2], *spare = w.s[3], *y0 = nullptr;
  double *r64 = w.r64, *acc = w.acc;
#define NM_MIX(KERN, ...)                                                                      \
  do {                                                                                         \
    if (v == 4)                                                                                \
      hipLaunchKernelGGL((KERN<4>), dim3(grid_for(lanes)), dim3(256), 0, st, __VA_ARGS__);      \
    else if (v == 2)                                                                           \
      hipLaunchKernelGGL((KERN<2>), dim3(grid_for(lanes)), dim3(256), 0, st, __VA_ARGS__);      \
    else                                                                                       \
      hipLaunchKernelGGL((KERN<1>), dim3(grid_for(lanes)), dim3(256), 0, st, __VA_ARGS__);      \
  } while (0)
  const int passes = cfg.mixP;
  NM_MIX(k_mix_first, (uint32_t)N, (uint32_t)wd, m64.mdinv, f, it, rhs, cur);
  for (int p = 0; p < passes; ++p) {
    for (int j = 1; j < cfg.mixK; ++j) {
      bool sampled = false;
      if (prof && j >= 2) prof->before(st, sampled);
      launch_cj_step<float>(N, wd, P->row_ptr.p, P->col.p, m32.ms, m32.mdinv, rhs, cur, prev, (float)cc.alpha[j - 1],
                            (float)cc.beta[j - 1], j == 1 ? 1 : 0, 0, prev, nullptr, nullptr, 0.f, 0.f, 0.f, 0, 0.f,
                            0.f, nullptr, nullptr, st, &tp);
      if (sampled) prof->after(st);
      std::swap(cur, prev);
    }
    if (p + 1 == passes) break;
    // cur: this pass's result; prev receives the next pass's first iterate
    NM_MIX(k_mix_resid, (uint32_t)N, (uint32_t)wd, P->row_ptr.p, P->col.p, m64.ms, m64.mdinv, p == 0 ? f : r64,
           p + 2 < passes ? r64 : nullptr, cur, p >= 2 ? acc : nullptr, p == 1 ? y0 : nullptr,
           p >= 1 ? acc : nullptr, it, rhs, prev);
    if (p == 0) {
      y0 = cur;  // kept until the next residual adds it to acc
      cur = prev;
      prev = spare;
    } else if (p == 1) {
      spare = y0;
      y0 = nullptr;
      std::swap(cur, prev);
    } else {
      std::swap(cur, prev);
    }
  }
  NM_MIX(k_mix_final, (uint32_t)N, (uint32_t)wd, passes >= 3 ? acc : nullptr, passes == 2 ? y0 : nullptr, cur,
         u.on ? 1 : 0, Z, (const double*)u.win, (const double*)u.wprev, u.a1, u.cs, u.a2, u.ymode, u.mu0, u.mu,
         (const double*)u.mu0c, (const double*)u.muc, (double*)u.wout, (double*)u.Y);
#undef NM_MIX
}

// z = S_M(A X) with one Chebyshev-Jacobi pass in T; either written to Z or
// consumed by the filter update u.  Work buffers: w.f, w.ya, w.yb [N][3b],
// the pressure buffers [n_p][b].
template <class T>
void b_apply_ws(const nm_pencil* P, int b, const T* X, T* Z, const Update& u, const ApplyCfg& cfg,
                const BWork<T>& w, hipStream_t st, KernelProf* prof = nullptr) {
  const int kM = cfg.kM, kP = cfg.kP;
  NM_REQUIRE(kM >= 2, NM_EINVAL, "the M solve needs at least 2 Chebyshev steps");
  auto m = mats<T>(P);
  ChebCoef cc = cheb_coef(P->ref.m_lo, P->ref.m_hi, kM);
  const MassPlan<T> tp = mass_plan<T>(P, b);
  a_apply<T>(P, b, X, w.f, w.ya, 1.0 / cc.theta, kP, w, st);
  const int64_t N = P->N;
  const int wd = 3 * b;
  T *cur = w.ya, *prev = w.yb;
  for (int j = 1; j < kM; ++j) {
    bool last = j == kM - 1;
    if (!last) {
      bool sampled = false;
      if (prof && j >= 2) prof->before(st, sampled);
      launch_cj_step<T>(N, wd, P->row_ptr.p, P->col.p, m.ms, m.mdinv, w.f, cur, prev, (T)cc.alpha[j - 1],
                        (T)cc.beta[j - 1], j == 1 ? 1 : 0, 0, prev, nullptr, nullptr, T(0), T(0), T(0), 0, T(0),
                        T(0), nullptr, nullptr, st, &tp);
      if (sampled) prof->after(st);
      std::swap(cur, prev);
    } else if (!u.on) {
      launch_cj_step<T>(N, wd, P->row_ptr.p, P->col.p, m.ms, m.mdinv, w.f, cur, prev, (T)cc.alpha[j - 1],
                        (T)cc.beta[j - 1], j == 1 ? 1 : 0, 0, Z, nullptr, nullptr, T(0), T(0), T(0), 0, T(0), T(0),
                        nullptr, nullptr, st, &tp);
    } else {
      launch_cj_step<T>(N, wd, P->row_ptr.p, P->col.p, m.ms, m.mdinv, w.f, cur, prev, (T)cc.alpha[j - 1],
                        (T)cc.beta[j - 1], j == 1 ? 1 : 0, 1, nullptr, (const T*)u.win, (const T*)u.wprev, (T)u.a1,
                        (T)u.cs, (T)u.a2, u.ymode, (T)u.mu0, (T)u.mu, (T*)u.wout, (T*)u.Y, st, &tp,
                        (const T*)u.mu0c, (const T*)u.muc);
    }
  }
}

// z = S_M(A X); either written to Z or consumed by the filter update u
template <class T>
void b_apply_impl(const nm_pencil* P, int b, const T* X, T* Z, const Update& u, const ApplyCfg& cfg,
                  FilterWork<T>& w, hipStream_t st, KernelProf* prof = nullptr) {
  if constexpr (std::is_same<T, double>::value) {
    if (cfg.mixP > 0) {
      NM_REQUIRE(cfg.kM >= 2, NM_EINVAL, "the M solve needs at least 2 Chebyshev steps");
      w.ensure_mixed(P, b);
      a_apply<double>(P, b, X, w.f.p, nullptr, 0.0, cfg.kP, w.bwork(), st);
      mass_solve_mixed(P, b, w.f.p, Z, u, cfg, MixBufs{w.ya.p, w.yb.p, {w.s0.p, w.s1.p, w.s2.p, w.s3.p}}, st, prof);
      return;
    }
  }
  b_apply_ws<T>(P, b, X, Z, u, cfg, w.bwork(), st, prof);
}

}  // namespace

int mass_kernel_kind(const nm_pencil* P, int b, bool fp32) {
  if (fp32) {
    const MassPlan<float> m = mass_plan<float>(P, b);
    return m.tile.on ? 2 : (m.group.on ? 1 : 0);
  }
  const MassPlan<double> m = mass_plan<double>(P, b);
  return m.tile.on ? 2 : (m.group.on ? 1 : 0);
}

int cheb_steps(double lo, double hi, double tol) {
  double kap = hi / lo;
  double r = (std::sqrt(kap) - 1.0) / (std::sqrt(kap) + 1.0);
  int k = (int)std::ceil(std::log(2.0 / tol) / std::log(1.0 / r));
  return std::max(k, 2);
}

template <class T>
void FilterWork<T>::ensure(const nm_pencil* P, int ncols) {
  if (b == ncols && f.p) return;
  b = ncols;
  size_t n = (size_t)P->N * 3 * ncols, np = (size_t)std::max<int64_t>(P->n_pres, 1) * ncols;
  x0.alloc(n); w0.alloc(n); w1.alloc(n); f.alloc(n); ya.alloc(n); yb.alloc(n);
  pt.alloc(np); ps.alloc(np); pa.alloc(np); pb.alloc(np);
}

template <class T>
void FilterWork<T>::ensure_mixed(const nm_pencil* P, int ncols) {
  ensure(P, ncols);
  const size_t n = (size_t)P->N * 3 * ncols;
  if (s0.n >= n && s0.p) return;
  s0.alloc(n); s1.alloc(n); s2.alloc(n); s3.alloc(n);
}

void set_mass_passes(nm_pencil* P, ApplyCfg& cfg, int passes, double mtol, int kM_pass, hipStream_t st) {
  cfg.mixP = 0;
  cfg.mixK = 0;
  if (passes == 0) return;
  NM_REQUIRE(passes >= 2 && passes <= 8, NM_EINVAL, "mass_passes must be 0 or 2..8");
  NM_REQUIRE(cfg.precision == 0, NM_EINVAL, "mass_passes applies to FP64 filters (precision 0)");
  NM_REQUIRE(kM_pass > 0 || mtol > 0, NM_EINVAL, "mass_passes needs a bound or a step count");
  cfg.mixP = passes;
  cfg.mixK = kM_pass > 0 ? kM_pass : cheb_steps(P->ref.m_lo, P->ref.m_hi, std::pow(mtol, 1.0 / passes));
  NM_REQUIRE(cfg.mixK >= 2, NM_EINVAL, "a mass-solve pass needs at least 2 steps");
  P->ensure_fp32(st);
}

template <class T>
void b_apply(const nm_pencil* P, int ncols, const T* X, T* Y, const ApplyCfg& cfg, FilterWork<T>& w,
             hipStream_t st) {
  check_block(3 * P->N, ncols);
  w.ensure(P, ncols);
  b_apply_impl<T>(P, ncols, X, Y, Update{}, cfg, w, st);
}

// Y = p(B) X, or ((B - l0)/s0) p(B) X when s0 != 0; p = sum_k mu_k T_k((t - c)/e).
// MUd (device, [m+1][ncols]) replaces mu by one series per column when set.
template <class T>
static void filter_run(const nm_pencil* P, const double* mu, const T* MUd, int m, double c, double e, double l0,
                       double s0, int ncols, const T* X, T* Y, const ApplyCfg& cfg, FilterWork<T>& w,
                       hipStream_t st) {
  check_block(3 * P->N, ncols);
  w.ensure(P, ncols);
  const int64_t n = P->N * 3 * ncols;
  if (m == 0 && s0 == 0.0) {
    LAUNCH(k_scale_copy<T>, n, st, n, (T)mu[0], X, Y);
    return;
  }
  T* bufs[2] = {w.w0.p, w.w1.p};
  const T* win = X;
  int nb = 0;  // next free buffer
  if (s0 != 0.0) {
    Update u;
    u.on = true; u.win = X; u.a1 = 1.0 / s0; u.cs = l0; u.a2 = 0.0; u.ymode = 0; u.wout = bufs[0];
    b_apply_impl<T>(P, ncols, X, nullptr, u, cfg, w, st, cfg.prof);
    win = bufs[0];
    nb = 1;
    if (m == 0) {
      LAUNCH(k_scale_copy<T>, n, st, n, (T)mu[0], win, Y);
      return;
    }
  }
  // step 1: W1 = (B W0 - c W0)/e ; Y = mu0 W0 + mu1 W1
  const T* wprev = nullptr;
  {
    Update u;
    u.on = true; u.win = win; u.a1 = 1.0 / e; u.cs = c; u.a2 = 0.0; u.ymode = 1;
    if (MUd) {
      u.mu0c = MUd;
      u.muc = MUd + ncols;
    } else {
      u.mu0 = mu[0];
      u.mu = mu[1];
    }
    u.wout = bufs[nb]; u.Y = Y;
    b_apply_impl<T>(P, ncols, win, nullptr, u, cfg, w, st, cfg.prof);
    wprev = win;
    win = bufs[nb];
    nb ^= 1;
  }
  for (int k = 2; k <= m; ++k) {
    // output buffer: the one holding wprev if it is a work buffer, else the free one
    T* out = (wprev == bufs[0] || wprev == bufs[1]) ? (T*)wprev : bufs[nb];
    Update u;
    u.on = true; u.win = win; u.wprev = wprev; u.a1 = 2.0 / e; u.cs = c; u.a2 = -1.0; u.ymode = 2;
    if (MUd)
      u.muc = MUd + (size_t)k * ncols;
    else
      u.mu = mu[k];
    u.wout = out; u.Y = Y;
    b_apply_impl<T>(P, ncols, win, nullptr, u, cfg, w, st, cfg.prof);
    wprev = win;
    win = out;
    nb = (out == bufs[0]) ? 1 : 0;
  }
}

template <class T>
void filter_apply(const nm_pencil* P, const double* mu, int m, double c, double e, double l0, double s0, int ncols,
                  const T* X, T* Y, const ApplyCfg& cfg, FilterWork<T>& w, hipStream_t st) {
  filter_run<T>(P, mu, nullptr, m, c, e, l0, s0, ncols, X, Y, cfg, w, st);
}

template <class T>
void filter_apply_cols(const nm_pencil* P, const double* mu_cols, int m, double c, double e, int ncols, const T* X,
                       T* Y, const ApplyCfg& cfg, FilterWork<T>& w, hipStream_t st) {
  NM_REQUIRE(m >= 1, NM_EINVAL, "per-column filters need degree >= 1");
  std::vector<T> h((size_t)(m + 1) * ncols);
  for (size_t i = 0; i < h.size(); ++i) h[i] = (T)mu_cols[i];
  w.ensure(P, ncols);
  if (w.mucols.n < h.size()) w.mucols.alloc(h.size());
  NM_HIP(hipMemcpyAsync(w.mucols.p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, st));
  filter_run<T>(P, nullptr, w.mucols.p, m, c, e, 0.0, 0.0, ncols, X, Y, cfg, w, st);
  // the host table must outlive the copy
  NM_HIP(hipStreamSynchronize(st));
}

// Density of states (kernel polynomial method): tau_k = (1/s) sum_v
// z_v . T_k((B - c)/e) z_v for k = 0..m from the s columns of Z (internal
// node order), by the filter's three-term recurrence (update fused into the
// mass solve, no series accumulation) with the column dots of each step
// reduced on the device in a fixed order.
void dos_traces(const nm_pencil* P, double lmin, double lmax, int m, int s, const double* Z, const ApplyCfg& cfg,
                hipStream_t st, double* tau, bool weighted) {
  check_block(3 * P->N, s);
  NM_REQUIRE(m >= 0 && lmax > lmin, NM_EINVAL, "need m >= 0 and lmax > lmin");
  const int64_t n = 3 * P->N;
  const double c = 0.5 * (lmax + lmin), e = 0.5 * (lmax - lmin);
  FilterWork<double> w;
  w.ensure(P, s);
  // weighted: the recurrence starts from B Z (traces of T_k((B - c)/e) B)
  DBuf<double> bz;
  if (weighted) {
    bz.alloc((size_t)n * s);
    b_apply_impl<double>(P, s, Z, bz.p, Update{}, cfg, w, st);
  }
  const double* start = weighted ? bz.p : Z;
  const int nblk = 512;
  DBuf<double> dots((size_t)(m + 1) * s), part((size_t)nblk * s);
  const int64_t rows_per = (n + nblk - 1) / nblk;
  auto coldot = [&](const double* W, int k) {
    hipLaunchKernelGGL(k_coldot_partial, dim3(nblk), dim3(256), 0, st, n, s, Z, s, W, s, rows_per, part.p);
    hipLaunchKernelGGL(k_coldot_final, dim3((s + 63) / 64), dim3(64), 0, st, nblk, s, part.p, dots.p + (size_t)k * s);
  };
  coldot(start, 0);
  double* bufs[2] = {w.w0.p, w.w1.p};
  const double* wprev = nullptr;
  const double* win = start;
  for (int k = 1; k <= m; ++k) {
    double* out = (wprev == bufs[0] || wprev == bufs[1]) ? (double*)wprev : (win == bufs[0] ? bufs[1] : bufs[0]);
    Update u;
    u.on = true;
    u.win = win;
    u.wprev = k >= 2 ? wprev : nullptr;
    u.a1 = (k == 1 ? 1.0 : 2.0) / e;
    u.cs = c;
    u.a2 = k == 1 ? 0.0 : -1.0;
    u.ymode = 0;
    u.wout = out;
    b_apply_impl<double>(P, s, win, nullptr, u, cfg, w, st);
    coldot(out, k);
    wprev = win;
    win = out;
  }
  std::vector<double> h((size_t)(m + 1) * s);
  NM_HIP(hipMemcpyAsync(h.data(), dots.p, 8 * h.size(), hipMemcpyDeviceToHost, st));
  NM_HIP(hipStreamSynchronize(st));
  for (int k = 0; k <= m; ++k) {
    double t = 0;
    for (int v = 0; v < s; ++v) t += h[(size_t)k * s + v];
    tau[k] = t / s;
  }
}

// Autotuning of the mass-solve step, the hot loop of every filter step: for
// block widths b in {8, 16, 32, 64} and every kernel -- one row per lane,
// row groups, and LDS tiles of 32 or 64 rows (the block size of the tiled
// sparse format) -- time `reps` middle Chebyshev-Jacobi steps with
// HIP events and keep the fastest per column.  Sets the pencil's kernel
// choice (and rebuilds its tiles at the winning size).
template <class T>
static void autotune_t(nm_pencil* P, hipStream_t st, int* best_b, double* best_us) {
  auto m = mats<T>(P);
  const int64_t N = P->N;
  const int bmax = 64, reps = 8;
  DBuf<T> f((size_t)N * 3 * bmax), y0((size_t)N * 3 * bmax), y1((size_t)N * 3 * bmax);
  NM_HIP(hipMemsetAsync(f.p, 0, f.bytes(), st));
  NM_HIP(hipMemsetAsync(y0.p, 0, y0.bytes(), st));
  NM_HIP(hipMemsetAsync(y1.p, 0, y1.bytes(), st));
  hipEvent_t e0, e1;
  NM_HIP(hipEventCreate(&e0));
  NM_HIP(hipEventCreate(&e1));
  double best = 1e300;
  const int rows0 = P->grp_rows;
  int bb = 16, bgrp = P->grouped, btile = 0, brows = rows0, bpersist = P->persist;
  // candidate kernels: (tile rows, grouped mode, rows per group); tile rows 0
  // = no tiles.  The row-group size is the block size of the grouped format
  // (rows x their column union, zero-padded): larger groups gather fewer
  // neighbour rows per output row but carry more coefficients and registers.
  struct Cand {
    int tr, grouped, rows, persist;
  };
  std::vector<Cand> cands = {{0, 0, 0, 0}};
  if (rows0 > 0)
    for (int r : {4, 8})
      for (int pe : {0, 1}) cands.push_back({0, 2, r, pe});
  for (int tr : {32, 64}) cands.push_back({tr, 0, 0, 0});
  const char* venv = getenv("NM_AUTOTUNE_VERBOSE");
  const bool verbose = venv && atoi(venv) != 0;
  for (const Cand& cd : cands) {
    if (cd.tr > 0) {
      build_tiles(P, st, cd.tr);
      if (P->tile_rows != cd.tr) continue;  // this tile size does not fit
    } else {
      P->tiled = 0;
    }
    if (cd.rows > 0 && P->grp_rows != cd.rows) {
      build_row_groups(P, st, cd.rows);
      if (P->grp_rows != cd.rows) continue;  // a group of this size does not fit the union sort
    }
    P->grouped = cd.grouped;
    P->persist = cd.persist;
    for (int b : {8, 16, 32, 64}) {
      const MassPlan<T> tp = mass_plan<T>(P, b);
      if (cd.tr > 0 && !tp.tile.on) continue;
      const int wd = 3 * b;
      auto step = [&]() {
        launch_cj_step<T>(N, wd, P->row_ptr.p, P->col.p, m.ms, m.mdinv, f.p, y0.p, y1.p, T(0.5), T(0.1), 0, 0, y1.p,
                          nullptr, nullptr, T(0), T(0), T(0), 0, T(0), T(0), nullptr, nullptr, st, &tp);
      };
      step();
      step();
      NM_HIP(hipEventRecord(e0, st));
      for (int r = 0; r < reps; ++r) step();
      NM_HIP(hipEventRecord(e1, st));
      NM_HIP(hipEventSynchronize(e1));
      float ms = 0;
      NM_HIP(hipEventElapsedTime(&ms, e0, e1));
      const double us = 1e3 * ms / reps / b;
      if (verbose)
        fprintf(stderr,
                "[autotune] %s b=%d kernel=%s tile_rows=%d group_rows=%d persistent=%d: %.1f us per step, %.3f us "
                "per column\n",
                sizeof(T) == 8 ? "fp64" : "fp32", b, tp.tile.on ? "tile" : (tp.group.on ? "group" : "row"), cd.tr,
                tp.group.on ? P->grp_rows : 0, tp.group.on && tp.group.persist ? 1 : 0, 1e3 * ms / reps, us);
      if (us < best) {
        best = us;
        bb = b;
        bgrp = cd.grouped;
        btile = cd.tr;
        brows = cd.rows > 0 ? cd.rows : rows0;
        bpersist = cd.persist;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (btile > 0) {
    build_tiles(P, st, btile);
  } else {
    P->tiled = 0;
  }
  if (brows > 0 && P->grp_rows != brows) build_row_groups(P, st, brows);
  P->grouped = bgrp;
  P->persist = bpersist;
  P->tuned_block = bb;
  P->tuned_tile = btile;
  *best_b = bb;
  *best_us = best;
}

void autotune(nm_pencil* P, int precision, hipStream_t st, int* best_b, double* best_us) {
  if (precision) {
    P->ensure_fp32(st);
    autotune_t<float>(P, st, best_b, best_us);
  } else {
    autotune_t<double>(P, st, best_b, best_us);
  }
  NM_HIP(hipStreamSynchronize(st));
}

template struct FilterWork<double>;
template struct FilterWork<float>;
template void filter_apply_cols<double>(const nm_pencil*, const double*, int, double, double, int, const double*,
                                        double*, const ApplyCfg&, FilterWork<double>&, hipStream_t);
template void filter_apply_cols<float>(const nm_pencil*, const double*, int, double, double, int, const float*,
                                       float*, const ApplyCfg&, FilterWork<float>&, hipStream_t);
template void b_apply<double>(const nm_pencil*, int, const double*, double*, const ApplyCfg&, FilterWork<double>&,
                              hipStream_t);
template void b_apply<float>(const nm_pencil*, int, const float*, float*, const ApplyCfg&, FilterWork<float>&,
                             hipStream_t);
template void filter_apply<double>(const nm_pencil*, const double*, int, double, double, double, double, int,
                                   const double*, double*, const ApplyCfg&, FilterWork<double>&, hipStream_t);
template void filter_apply<float>(const nm_pencil*, const double*, int, double, double, double, double, int,
                                  const float*, float*, const ApplyCfg&, FilterWork<float>&, hipStream_t);

// Y = op(X) with caller-provided work buffers (see op_work_elems); stream
// ordered, no synchronisation and no allocation.  The mixed-precision mass
// solve (cfg.mixP) is not available here.
template <class T>
static void apply_op_ws_t(const nm_pencil* P, int op, int b, const void* Xv, void* Yv, const ApplyCfg& cfg,
                          const BWork<T>& w, hipStream_t st) {
  const T* X = (const T*)Xv;
  T* Y = (T*)Yv;
  auto m = mats<T>(P);
  const int64_t N = P->N, NP = P->n_pres;
  const int wd = 3 * b;
  switch (op) {
    case NM_OP_AG:
      launch_apply_ag<T>(N, b, P->row_ptr.p, P->col.p, m.ag, X, nullptr, nullptr, nullptr, nullptr, Y, nullptr, T(0),
                         nullptr, st);
      break;
    case NM_OP_M:
      launch_spmm_scalar<T>(N, wd, P->row_ptr.p, P->col.p, m.ms, X, Y, st);
      break;
    case NM_OP_R:
      LAUNCH(k_spmm_coriolis<T>, N * wd, st, N, b, P->row_ptr.p, P->col.p, m.ms, (T)P->omega[0], (T)P->omega[1],
             (T)P->omega[2], X, Y);
      break;
    case NM_OP_KP:
      NM_REQUIRE(NP > 0, NM_EINVAL, "pencil has no pressure unknowns");
      launch_spmm_scalar<T>(NP, b, P->kp_ptr.p, P->kp_col.p, m.kp, X, Y, st);
      break;
    case NM_OP_EG:
      NM_REQUIRE(NP > 0, NM_EINVAL, "pencil has no pressure unknowns");
      LAUNCH(k_eg<T>, N * wd, st, N, b, P->eg_ptr.p, P->eg_col.p, m.eg, X, Y);
      break;
    case NM_OP_EGT:
      NM_REQUIRE(NP > 0, NM_EINVAL, "pencil has no pressure unknowns");
      LAUNCH(k_egt<T>, NP * b, st, NP, b, P->egt_ptr.p, P->egt_col.p, m.egt, X, Y);
      break;
    case NM_OP_KPINV: {
      NM_REQUIRE(NP > 0, NM_EINVAL, "pencil has no pressure unknowns");
      NM_REQUIRE(cfg.kP >= 1, NM_EINVAL, "kP must be >= 1");
      T* r = kp_solve<T>(P, b, X, cfg.kP, w.pa, w.pb, st);
      NM_HIP(hipMemcpyAsync(Y, r, NP * b * sizeof(T), hipMemcpyDeviceToDevice, st));
      break;
    }
    case NM_OP_A:
      a_apply<T>(P, b, X, Y, nullptr, 0.0, cfg.kP, w, st);
      break;
    case NM_OP_MINV: {
      NM_REQUIRE(cfg.kM >= 2, NM_EINVAL, "kM must be >= 2");
      ChebCoef cc = cheb_coef(P->ref.m_lo, P->ref.m_hi, cfg.kM);
      const MassPlan<T> tp = mass_plan<T>(P, b);
      launch_cj_first<T>(N, wd, m.mdinv, X, (T)(1.0 / cc.theta), w.ya, st);
      T *cur = w.ya, *prev = w.yb;
      for (int j = 1; j < cfg.kM; ++j) {
        T* out = j == cfg.kM - 1 ? Y : prev;
        launch_cj_step<T>(N, wd, P->row_ptr.p, P->col.p, m.ms, m.mdinv, X, cur, prev, (T)cc.alpha[j - 1],
                          (T)cc.beta[j - 1], j == 1 ? 1 : 0, 0, out, nullptr, nullptr, T(0), T(0), T(0), 0, T(0),
                          T(0), nullptr, nullptr, st, &tp);
        std::swap(cur, prev);
      }
      break;
    }
    case NM_OP_B:
      b_apply_ws<T>(P, b, X, Y, Update{}, cfg, w, st);
      break;
    default:
      throw Error(NM_EINVAL, "unknown operator " + std::to_string(op));
  }
  NM_HIP(hipGetLastError());
}

template <class T>
static void apply_op_t(const nm_pencil* P, int op, int b, const void* Xv, void* Yv, const ApplyCfg& cfg,
                       hipStream_t st) {
  if constexpr (std::is_same<T, double>::value) {
    if (op == NM_OP_MINV && cfg.mixP > 0) {
      const size_t n = (size_t)P->N * 3 * b;
      DBuf<double> r64(n), acc(n);
      DBuf<float> s0(n), s1(n), s2(n), s3(n);
      mass_solve_mixed(P, b, (const double*)Xv, (double*)Yv, Update{}, cfg,
                       MixBufs{r64.p, acc.p, {s0.p, s1.p, s2.p, s3.p}}, st, nullptr);
      NM_HIP(hipStreamSynchronize(st));
      NM_HIP(hipGetLastError());
      return;
    }
    if (op == NM_OP_B && cfg.mixP > 0) {
      FilterWork<double> fw;
      b_apply<double>(P, b, (const double*)Xv, (double*)Yv, cfg, fw, st);
      NM_HIP(hipStreamSynchronize(st));
      return;
    }
  }
  OpWorkElems need = op_work_elems(P, op, b);
  DBuf<T> vec(need.vec * need.nvec), pres(need.pres * need.npres);
  BWork<T> w;
  T* v[3] = {nullptr, nullptr, nullptr};
  for (int i = 0; i < need.nvec; ++i) v[i] = vec.p + (size_t)i * need.vec;
  if (need.nvec == 3) {
    w.f = v[0]; w.ya = v[1]; w.yb = v[2];
  } else if (need.nvec == 2) {
    w.ya = v[0]; w.yb = v[1];
  }
  T* q[3] = {nullptr, nullptr, nullptr};
  for (int i = 0; i < need.npres; ++i) q[i] = pres.p + (size_t)i * need.pres;
  if (need.npres == 3) {
    w.pt = q[0]; w.pa = q[1]; w.pb = q[2];
  } else if (need.npres == 2) {
    w.pa = q[0]; w.pb = q[1];
  }
  apply_op_ws_t<T>(P, op, b, Xv, Yv, cfg, w, st);
  NM_HIP(hipStreamSynchronize(st));
}

template <class T>
__global__ void k_permute_rows(int64_t rows, int w, const T* __restrict__ src, T* __restrict__ dst,
                               const int32_t* __restrict__ map) {
  int64_t g = (int64_t)nm_xcd_block() * blockDim.x + threadIdx.x;
  if (g >= rows * w) return;
  int64_t r = g / w;
  int e = (int)(g - r * w);
  dst[g] = src[(int64_t)map[r] * w + e];
}

void permute_rows(int64_t rows, int w, const void* src, void* dst, const int32_t* map, int elem_bytes,
                  hipStream_t st) {
  if (elem_bytes == 8)
    LAUNCH(k_permute_rows<double>, rows * w, st, rows, w, (const double*)src, (double*)dst, map);
  else
    LAUNCH(k_permute_rows<float>, rows * w, st, rows, w, (const float*)src, (float*)dst, map);
}

void api_apply(const nm_pencil* P, int op, int ncols, const void* X, void* Y, const ApplyCfg& cfg,
               hipStream_t st) {
  check_block(3 * P->N, ncols);
  const int eb = cfg.precision == 1 ? 4 : 8;
  const bool in_disp = !(op == NM_OP_KP || op == NM_OP_EG || op == NM_OP_KPINV);
  const bool out_disp = !(op == NM_OP_KP || op == NM_OP_EGT || op == NM_OP_KPINV);
  const int64_t N = P->N, w = 3 * (int64_t)ncols;
  DBuf<char> xi, yi;
  const void* xin = X;
  void* yout = Y;
  if (in_disp) {
    xi.alloc((size_t)N * w * eb);
    permute_rows(N, (int)w, X, xi.p, P->iperm.p, eb, st);
    xin = xi.p;
  }
  if (out_disp) {
    yi.alloc((size_t)N * w * eb);
    yout = yi.p;
  }
  apply_op(P, op, ncols, xin, yout, cfg, st);
  if (out_disp) permute_rows(N, (int)w, yi.p, Y, P->perm.p, eb, st);
  NM_HIP(hipStreamSynchronize(st));
}

OpWorkElems op_work_elems(const nm_pencil* P, int op, int b) {
  OpWorkElems e;
  const size_t vec = (size_t)P->N * 3 * b, pres = (size_t)std::max<int64_t>(P->n_pres, 1) * b;
  switch (op) {
    case NM_OP_KPINV:
      e.pres = pres; e.npres = 2;
      break;
    case NM_OP_A:
      e.pres = pres; e.npres = 3;
      break;
    case NM_OP_MINV:
      e.vec = vec; e.nvec = 2;
      break;
    case NM_OP_B:
      e.vec = vec; e.nvec = 3; e.pres = pres; e.npres = 3;
      break;
    default:
      break;
  }
  return e;
}

void apply_op_ws(const nm_pencil* P, int op, int ncols, const void* X, void* Y, const ApplyCfg& cfg, void* work,
                 hipStream_t st) {
  check_block(3 * P->N, ncols);
  NM_REQUIRE(cfg.mixP == 0, NM_EINVAL, "the mixed-precision mass solve needs its own work buffers");
  const OpWorkElems need = op_work_elems(P, op, ncols);
  auto carve = [&](auto* base, auto& w) {
    using T = std::remove_pointer_t<decltype(base)>;
    T* v = base;
    T* a[3] = {nullptr, nullptr, nullptr};
    for (int i = 0; i < need.nvec; ++i) a[i] = v + (size_t)i * need.vec;
    T* pr = v + (size_t)need.nvec * need.vec;
    T* b[3] = {nullptr, nullptr, nullptr};
    for (int i = 0; i < need.npres; ++i) b[i] = pr + (size_t)i * need.pres;
    if (need.nvec == 3) { w.f = a[0]; w.ya = a[1]; w.yb = a[2]; }
    if (need.nvec == 2) { w.ya = a[0]; w.yb = a[1]; }
    if (need.npres == 3) { w.pt = b[0]; w.pa = b[1]; w.pb = b[2]; }
    if (need.npres == 2) { w.pa = b[0]; w.pb = b[1]; }
  };
  if (cfg.precision == 1) {
    NM_REQUIRE(P->ms32.p, NM_EINVAL, "FP32 operators before the pencil's FP32 matrices exist");
    BWork<float> w;
    carve((float*)work, w);
    apply_op_ws_t<float>(P, op, ncols, X, Y, cfg, w, st);
  } else {
    BWork<double> w;
    carve((double*)work, w);
    apply_op_ws_t<double>(P, op, ncols, X, Y, cfg, w, st);
  }
}

void apply_op(const nm_pencil* P, int op, int ncols, const void* X, void* Y, const ApplyCfg& cfg, hipStream_t st) {
  check_block(3 * P->N, ncols);
  if (cfg.precision == 1) {
    const_cast<nm_pencil*>(P)->ensure_fp32(st);
    apply_op_t<float>(P, op, ncols, X, Y, cfg, st);
  } else {
    apply_op_t<double>(P, op, ncols, X, Y, cfg, st);
  }
}

void col_dots(int64_t rows, int ncols, const double* X, int ldx, const double* Y, int ldy, double* out,
              hipStream_t st) {
  const int nblk = 512;
  int64_t rows_per = (rows + nblk - 1) / nblk;
  DBuf<double> part((size_t)nblk * ncols);
  hipLaunchKernelGGL(k_coldot_partial, dim3(nblk), dim3(256), 0, st, rows, ncols, X, ldx, Y, ldy, rows_per, part.p);
  hipLaunchKernelGGL(k_coldot_final, dim3((ncols + 63) / 64), dim3(64), 0, st, nblk, ncols, part.p, out);
  NM_HIP(hipStreamSynchronize(st));
}

void KernelProf::before(hipStream_t st, bool& sampled) {
  sampled = (launches++ % every) == 0;
  if (!sampled) return;
  if (used + 2 > (int)pool.size()) {
    if (pool.size() < 512) {
      for (int i = 0; i < 64; ++i) {
        hipEvent_t e;
        NM_HIP(hipEventCreate(&e));
        pool.push_back(e);
      }
    } else {
      harvest();
    }
  }
  NM_HIP(hipEventRecord(pool[used], st));
}
void KernelProf::after(hipStream_t st) {
  NM_HIP(hipEventRecord(pool[used + 1], st));
  used += 2;
}
void KernelProf::harvest() {
  for (int i = 0; i + 1 < used; i += 2) {
    NM_HIP(hipEventSynchronize(pool[i + 1]));
    float t = 0.f;
    NM_HIP(hipEventElapsedTime(&t, pool[i], pool[i + 1]));
    ms += t;
    ++samples;
  }
  used = 0;
}
KernelProf::~KernelProf() {
  for (auto e : pool) (void)hipEventDestroy(e);
}

void convert_f64_f32(int64_t n, const double* a, float* b, hipStream_t st) {
  LAUNCH(k_f64_f32, n, st, n, a, b);
}
void convert_f32_f64(int64_t n, const float* a, double* b, hipStream_t st) {
  LAUNCH(k_f32_f64, n, st, n, a, b);
}

}  // namespace nm

void nm_pencil::ensure_fp32(hipStream_t st) {
  std::lock_guard<std::mutex> lk(fp32_mx);
  if (ms32.p) return;
  auto cv = [&](const nm::DBuf<double>& a, nm::DBuf<float>& b) {
    b.alloc(std::max<size_t>(a.n, 1));
    if (a.n) nm::convert_f64_f32((int64_t)a.n, a.p, b.p, st);
  };
  cv(ag, ag32); cv(ms, ms32); cv(mdinv, mdinv32);
  cv(kp, kp32); cv(kpdinv, kpdinv32); cv(eg_val, eg_val32); cv(egt_val, egt_val32);
  if (grp_rows > 0) cv(grp_coef, grp_coef32);
  NM_HIP(hipStreamSynchronize(st));
}
