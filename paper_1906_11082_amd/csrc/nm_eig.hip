// Polynomial-filtered block Lanczos for the Cowling pencil (Sec. 6.1 of the
// paper: polynomial filtering on [f1, f2], A and M accessed through
// products; filter and Lanczos details follow the cited EVSL approach).
//
//  * spectrum bounds of B = M^{-1} A: a short Lanczos in the M-inner product;
//  * filter: Jackson-damped Chebyshev series of the window indicator,
//    optionally times (B - lambda_0)/s, which annihilates an exactly
//    degenerate null space (rigid motions, the fluid kernel of the
//    Cowling operator with N^2 = 0) without resolving the gap below the
//    window;
//  * block Krylov on p(B) in the M-inner product with full, twice-iterated
//    block Gram-Schmidt and Cholesky QR (twice), keeping A V;
//  * Rayleigh-Ritz with the original pencil (A, M) on the basis; stop when
//    every Ritz pair in the window has residual <= tol, their count is
//    stable and every Ritz value of p(B) above the filter's window level
//    has converged.
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <cmath>
#include <numeric>

#include "nm_internal.h"

namespace nm {

// ------------------------------------------------------------ filter design
void jackson_chebyshev(double a, double b, double lmin, double lmax, int m, double* mu) {
  const double c = 0.5 * (lmax + lmin), e = 0.5 * (lmax - lmin);
  double al = std::min(1.0, std::max(-1.0, (a - c) / e));
  double be = std::min(1.0, std::max(-1.0, (b - c) / e));
  const double ta = std::acos(al), tb = std::acos(be);
  const double th = M_PI / (m + 2);
  for (int k = 0; k <= m; ++k) {
    double gam = k == 0 ? (ta - tb) / M_PI : 2.0 * (std::sin(k * ta) - std::sin(k * tb)) / (M_PI * k);
    double jac = ((1.0 - (double)k / (m + 2)) * std::sin(th) * std::cos(k * th) +
                  std::cos(th) * std::sin(k * th) / (m + 2)) / std::sin(th);
    mu[k] = gam * jac;
  }
}

double cheb_eval(const double* mu, int m, double t) {
  double t0 = 1.0, t1 = t, s = mu[0] + (m >= 1 ? mu[1] * t : 0.0);
  for (int k = 2; k <= m; ++k) {
    double t2 = 2.0 * t * t1 - t0;
    s += mu[k] * t2;
    t0 = t1;
    t1 = t2;
  }
  return s;
}

namespace {
double filter_value(const std::vector<double>& mu, int m, double c, double e, double lam, bool null, double s0) {
  double p = cheb_eval(mu.data(), m, std::min(1.0, std::max(-1.0, (lam - c) / e)));
  return null ? p * lam / s0 : p;
}
}  // namespace

// Smallest degree (on a 15 % ladder) whose filter stays below 1 % of its
// window-edge level beyond the guard point b (1 + guard); lower side:
//   mode 0  no requirement below a.  For the Cowling pencil with N^2 = 0 the
//           spectrum below the window is the exactly degenerate fluid null
//           space (plus rigid motions): a Krylov method sees a degenerate
//           eigenvalue as one direction per start vector, so it needs no
//           damping; the few other low modes converge as unwanted pairs.
//   mode 1  the same bound below a - guard (a - lmin);
//   mode 2  the filter is multiplied by lambda / b (null factor).
//   mode 3  spectrum slices: two-sided, with guard points a - guard (b - a) and
//           b + guard (b - a) (bands proportional to the slice's width), so
//           that the slices of one window each damp the others' eigenvalues.
int choose_degree(double a, double b, double lmin, double lmax, double guard, int mode) {
  if (guard <= 0) guard = 1.0;
  const bool null = mode == 2;
  const double c = 0.5 * (lmax + lmin), e = 0.5 * (lmax - lmin);
  const double bg = mode == 3 ? b + guard * (b - a) : b * (1.0 + guard);
  const double ag = mode == 3 ? a - guard * (b - a) : a - guard * std::max(a - lmin, 0.0);
  const double s0 = null ? b : 0.0;
  std::vector<double> mu;
  for (double md = 8; md < 20000; md *= 1.15) {
    int m = (int)md;
    mu.resize(m + 1);
    jackson_chebyshev(a, b, lmin, lmax, m, mu.data());
    double pa = filter_value(mu, m, c, e, a, null, s0), pb = filter_value(mu, m, c, e, b, null, s0);
    double lev = std::min(pa, pb);
    if (!(lev > 0)) continue;
    bool ok = true;
    // sample uniformly in angle, which resolves the polynomial's oscillations
    const int ns = 4 * m + 64;
    double th_hi = std::acos(std::min(1.0, std::max(-1.0, (bg - c) / e)));
    for (int i = 0; i <= ns && ok && bg < lmax; ++i) {
      double th = th_hi * i / ns;
      double lam = c + e * std::cos(th);
      if (std::fabs(filter_value(mu, m, c, e, lam, null, s0)) > 0.01 * lev) ok = false;
    }
    if ((mode == 1 || mode == 3) && ag > lmin) {
      double th_lo = std::acos(std::min(1.0, std::max(-1.0, (ag - c) / e)));
      for (int i = 0; i <= ns && ok; ++i) {
        double th = th_lo + (M_PI - th_lo) * i / ns;
        double lam = c + e * std::cos(th);
        if (std::fabs(filter_value(mu, m, c, e, lam, null, s0)) > 0.01 * lev) ok = false;
      }
    }
    if (ok) return m;
  }
  throw Error(NM_EINVAL, "no filter degree below 20000 separates the window");
}

namespace {

__device__ __forceinline__ int64_t gtid() { return nm_xcd_block() * blockDim.x + threadIdx.x; }

// counter-based N(0,1): splitmix64 hash of (seed, column, row), Box-Muller
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__global__ void k_randn(int64_t rows, int nc, int ld, uint64_t seed, int64_t col0, double* X) {
  int64_t g = gtid();
  if (g >= rows * nc) return;
  int64_t r = g / nc;
  int v = (int)(g % nc);
  uint64_t h = mix64(mix64(seed ^ mix64((uint64_t)(col0 + v) * 0x632BE59BD9B4E019ull)) ^ (uint64_t)r);
  uint64_t h2 = mix64(h);
  double u1 = ((h >> 11) + 1.0) * (1.0 / 9007199254740993.0);
  double u2 = (h2 >> 11) * (1.0 / 9007199254740992.0);
  X[r * ld + v] = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

__global__ void k_sub_scaled_cols(int64_t rows, int nc, const double* __restrict__ AX,
                                  const double* __restrict__ MX, const double* __restrict__ th,
                                  double* __restrict__ R) {
  int64_t g = gtid();
  if (g >= rows * nc) return;
  int v = (int)(g % nc);
  R[g] = AX[g] - th[v] * MX[g];
}

// per column: index of the entry of largest magnitude -> sign
__global__ void k_col_sign(int64_t rows, int nc, const double* __restrict__ X, double* __restrict__ sgn) {
  int v = blockIdx.x;
  __shared__ double bv[256];
  double best = 0.0, val = 0.0;
  for (int64_t r = threadIdx.x; r < rows; r += blockDim.x) {
    double x = X[r * nc + v];
    if (fabs(x) > best) { best = fabs(x); val = x; }
  }
  // reduce by magnitude, ties resolved toward the smaller thread (row order)
  __shared__ double bm[256];
  bm[threadIdx.x] = best;
  bv[threadIdx.x] = val;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o && bm[threadIdx.x + o] > bm[threadIdx.x]) {
      bm[threadIdx.x] = bm[threadIdx.x + o];
      bv[threadIdx.x] = bv[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) sgn[v] = bv[0] < 0 ? -1.0 : 1.0;
}
__global__ void k_scale_cols(int64_t rows, int nc, const double* __restrict__ s, double* __restrict__ X) {
  int64_t g = gtid();
  if (g >= rows * nc) return;
  X[g] *= s[g % nc];
}

struct Blas {
  rocblas_handle h;  // small dense products (k x k) and the dense eigensolver
  hipStream_t st;
  DBuf<double> ws;  // row-chunk partial products of tn
  // row-major helpers on the FP64 matrix cores (nm_gemm.hip)
  // C[K][q] (col-major K x q, ld K) = A^T B, A row-major [n][*] (ld lda, first K cols), B row-major [n][*] (q cols)
  void tn(int64_t n, int K, int q, const double* A, int lda, const double* B, int ldb, double* C) {
    gemm_tn(n, K, q, A, lda, B, ldb, C, ws, st);
  }
  // D (row-major [n][q], ld ldd) = alpha * A (row-major [n][K], ld lda) * C (col-major K x q, ld ldc) + beta * D
  void nn(int64_t n, int K, int q, double alpha, const double* A, int lda, const double* C, int ldc, double beta,
          double* D, int ldd) {
    gemm_nn(n, K, q, alpha, A, lda, C, ldc, beta, D, ldd, st);
  }
};

void chol_upper(int b, std::vector<double>& G, bool& ok) {
  // in place: G (col-major b x b, symmetric) -> R upper with G = R^T R
  ok = true;
  for (int j = 0; j < b; ++j) {
    double s = G[j + j * b];
    for (int k = 0; k < j; ++k) s -= G[k + j * b] * G[k + j * b];
    if (!(s > 0)) { ok = false; return; }
    double r = std::sqrt(s);
    G[j + j * b] = r;
    for (int i = j + 1; i < b; ++i) {
      double t = G[j + i * b];
      for (int k = 0; k < j; ++k) t -= G[k + j * b] * G[k + i * b];
      G[j + i * b] = t / r;
    }
    for (int i = j + 1; i < b; ++i) G[i + j * b] = 0.0;
  }
}

void upper_inverse(int b, const std::vector<double>& R, std::vector<double>& Ri) {
  Ri.assign(b * b, 0.0);
  for (int j = 0; j < b; ++j) {
    Ri[j + j * b] = 1.0 / R[j + j * b];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0;
      for (int k = i + 1; k <= j; ++k) s += R[i + k * b] * Ri[k + j * b];
      Ri[i + j * b] = -s / R[i + i * b];
    }
  }
}

// device -> host copy ordered on stream st (a plain hipMemcpy runs on the null
// stream, which would serialise concurrent solves on their own streams)
void d2h_sync(double* h, const double* d, size_t count, hipStream_t st) {
  NM_HIP(hipMemcpyAsync(h, d, 8 * count, hipMemcpyDeviceToHost, st));
  NM_HIP(hipStreamSynchronize(st));
}

struct Timer {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double s() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

}  // namespace

namespace {

// w_p = sum over the displacement DOFs (j, b) of |E_G[(j, b), p]| / sqrt(M_s,jj)
__global__ void k_bound_w(int64_t np, const int32_t* __restrict__ tp, const int32_t* __restrict__ tc,
                          const double* __restrict__ tv, const double* __restrict__ mdinv, double* __restrict__ w) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  double s = 0.0;
  for (int32_t k = tp[p]; k < tp[p + 1]; ++k)
    s += (fabs(tv[3 * (int64_t)k]) + fabs(tv[3 * (int64_t)k + 1]) + fabs(tv[3 * (int64_t)k + 2])) * sqrt(mdinv[tc[k]]);
  w[p] = s;
}

// per node i, the largest over its three DOFs a of the Gershgorin row sum of
// D^{-1/2} A_G D^{-1/2} plus the row bound of D^{-1/2} E_G D_p^{-1} E_G^T D^{-1/2} / theta_p
__global__ void k_bound_rows(int64_t N, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                             const double* __restrict__ ag, const double* __restrict__ mdinv,
                             const int32_t* __restrict__ ep, const int32_t* __restrict__ ec,
                             const double* __restrict__ ev, const double* __restrict__ w,
                             const double* __restrict__ kpdinv, double inv_theta_p, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double si = sqrt(mdinv[i]);
  double best = 0.0;
  for (int a = 0; a < 3; ++a) {
    double g = 0.0;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      const double* blk = ag + 9 * (int64_t)k + 3 * a;
      g += (fabs(blk[0]) + fabs(blk[1]) + fabs(blk[2])) * si * sqrt(mdinv[col[k]]);
    }
    double e = 0.0;
    if (ep)
      for (int32_t k = ep[i]; k < ep[i + 1]; ++k) e += fabs(ev[3 * (int64_t)k + a]) * w[ec[k]] * kpdinv[ec[k]] * si;
    best = fmax(best, g + inv_theta_p * e);
  }
  out[i] = best;
}

}  // namespace

// A bound that holds for every eigenvalue of the Cowling pencil (A, M),
// A = A_G + E_G K_p^{-1} E_G^T, with D = diag(M):
//   x^T M x >= theta_M x^T D x  (theta_M the reference element's lower Jacobi
//   bound of M, valid for the assembled matrix), K_p >= theta_p D_p likewise,
//   so lambda_max <= [max row sum of |D^{-1/2} A_G D^{-1/2}|
//                     + max row bound of D^{-1/2} E_G D_p^{-1} E_G^T D^{-1/2} / theta_p] / theta_M
// (Gershgorin; the Schur row bound from sum_p |E_ip| w_p / D_p,pp).  Looser
// than the Lanczos estimate, so the filter is built on the estimate and the
// bound serves the blow-up restart.  Without the self-gravitation term.
double lmax_rigorous(const nm_pencil* P, hipStream_t st) {
  const int64_t N = P->N, np = P->n_pres;
  DBuf<double> rows(N);
  DBuf<double> w(std::max<int64_t>(np, 1));
  const bool fl = np > 0;
  if (fl)
    hipLaunchKernelGGL(k_bound_w, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, np, P->egt_ptr.p,
                       P->egt_col.p, P->egt_val.p, P->mdinv.p, w.p);
  hipLaunchKernelGGL(k_bound_rows, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, N, P->row_ptr.p, P->col.p,
                     P->ag.p, P->mdinv.p, fl ? P->eg_ptr.p : nullptr, fl ? P->eg_col.p : nullptr,
                     fl ? P->eg_val.p : nullptr, w.p, fl ? P->kpdinv.p : nullptr, fl ? 1.0 / P->ref.p_lo : 0.0,
                     rows.p);
  NM_HIP(hipGetLastError());
  std::vector<double> h(N);
  NM_HIP(hipMemcpyAsync(h.data(), rows.p, 8 * N, hipMemcpyDeviceToHost, st));
  NM_HIP(hipStreamSynchronize(st));
  double mx = 0.0;
  for (double v : h) mx = std::max(mx, v);
  return mx / P->ref.m_lo;
}


// Bounds of spec(M^{-1} A) from `steps` Lanczos steps in the M-inner
// product (full reorthogonalisation): lmax = 1.01 (theta_max + |beta s|),
// a safe upper bound once the top Ritz value has converged;
// lmin = min(0, theta_min) - min(|beta s|_min, |theta_min| + 1e-12): the
// bottom of the spectrum (rigid motions, the fluid null space) is dense and
// converges slowly, and an estimate a little above the true minimum only
// lets the Chebyshev polynomials grow mildly there.
void spectrum_bounds(const nm_pencil* P, int steps_req, uint64_t seed, hipStream_t st, double* lmin_out,
                     double* lmax_out) {
  const int64_t n = 3 * P->N;
  const int steps = (int)std::min<int64_t>(steps_req, n - 1);
  NM_REQUIRE(steps >= 2, NM_EINVAL, "problem too small for spectrum bounds");
  Blas bl{P->blas, st, {}};
  NM_BLAS(rocblas_set_stream(bl.h, st));
  NM_BLAS(rocblas_set_pointer_mode(bl.h, rocblas_pointer_mode_host));
  ApplyCfg bc;
  bc.precision = 0;
  bc.kM = cheb_steps(P->ref.m_lo, P->ref.m_hi, 1e-12);
  bc.kP = cheb_steps(P->ref.p_lo, P->ref.p_hi, 1e-13);
  FilterWork<double> w1;
  DBuf<double> Vl((size_t)n * (steps + 1)), z(n), mz(n), dots(std::max(steps + 1, 2));
  hipLaunchKernelGGL(k_randn, dim3(grid_for(n)), dim3(256), 0, st, n, 1, 1, seed, 0, Vl.p);
  std::vector<double> al, be;
  const double one = 1.0, zero = 0.0, m1 = -1.0;
  auto mnorm = [&](const double* v) {
    apply_op(P, NM_OP_M, 1, v, mz.p, bc, st);
    double d;
    col_dots(n, 1, v, 1, mz.p, 1, dots.p, st);
    d2h_sync(&d, dots.p, 1, st);
    return std::sqrt(std::max(d, 0.0));
  };
  double inv = 1.0 / mnorm(Vl.p);
  NM_BLAS(rocblas_dscal(bl.h, (rocblas_int)n, &inv, Vl.p, 1));
  for (int k = 0; k < steps; ++k) {
    double* v = Vl.p + (size_t)k * n;
    b_apply<double>(P, 1, v, z.p, bc, w1, st);
    for (int pass = 0; pass < 2; ++pass) {
      apply_op(P, NM_OP_M, 1, z.p, mz.p, bc, st);
      std::vector<double> h(k + 1);
      NM_BLAS(rocblas_dgemv(bl.h, rocblas_operation_transpose, (rocblas_int)n, k + 1, &one, Vl.p, (rocblas_int)n,
                            mz.p, 1, &zero, dots.p, 1));
      NM_HIP(hipMemcpyAsync(h.data(), dots.p, 8 * (k + 1), hipMemcpyDeviceToHost, st));
      NM_HIP(hipStreamSynchronize(st));
      if (pass == 0) al.push_back(h[k]);
      else al.back() += h[k];
      NM_BLAS(rocblas_dgemv(bl.h, rocblas_operation_none, (rocblas_int)n, k + 1, &m1, Vl.p, (rocblas_int)n, dots.p, 1,
                            &one, z.p, 1));
    }
    double bt = mnorm(z.p);
    be.push_back(bt);
    if (!(bt > 1e-12 * std::fabs(al.back())) || !std::isfinite(bt)) break;
    double ib = 1.0 / bt;
    NM_HIP(hipMemcpyAsync(Vl.p + (size_t)(k + 1) * n, z.p, 8 * n, hipMemcpyDeviceToDevice, st));
    NM_BLAS(rocblas_dscal(bl.h, (rocblas_int)n, &ib, Vl.p + (size_t)(k + 1) * n, 1));
  }
  int m = (int)al.size();
  std::vector<double> Tm(m * m, 0.0), th, S;
  for (int i = 0; i < m; ++i) {
    Tm[i + i * m] = al[i];
    if (i + 1 < m) Tm[i + (i + 1) * m] = Tm[(i + 1) + i * m] = be[i];
  }
  jacobi_eig(m, Tm, th, &S);
  double rmax = std::fabs(be[m - 1] * S[(m - 1) + (m - 1) * m]);
  double rmin = std::fabs(be[m - 1] * S[(m - 1) + 0 * m]);
  NM_REQUIRE(std::isfinite(th[m - 1]) && std::isfinite(rmax), NM_ENOCONV, "non-finite Lanczos bounds");
  *lmax_out = (th[m - 1] + rmax) * 1.01;
  *lmin_out = std::min(0.0, th[0]) - std::min(rmin, std::fabs(th[0]) + 1e-12);
}

// block width: given, else the autotuner's (at most nev / 4, in multiples of 8), else 16
int solve_block_width(const nm_pencil* P, const nm_eig_opts& o, int nev) {
  const int bs = o.block > 0 ? o.block
                             : (P->tuned_block > 0 ? std::min(P->tuned_block, std::max(8, nev / 4 / 8 * 8)) : 16);
  return (int)std::min<int64_t>(bs, 3 * P->N);
}

namespace {
// the filtered vectors grew without bound: an eigenvalue lies above the
// interval the Chebyshev polynomials were mapped to (lambda_max too small)
struct FilterBlowUp : Error {
  double lmin, lmax;
  FilterBlowUp(double lo, double hi)
      : Error(NM_ENOCONV, "filter blow-up: the spectrum bound lambda_max is too small"), lmin(lo), lmax(hi) {}
};
}  // namespace

static void filtered_eig_once(const nm_pencil* P, double a, double b, int nev, double tol, const nm_eig_opts& o,
                              nm_eig_result** out, BatchSeat* seat, rocblas_handle blas);

// A blow-up means the bound lambda_max was below the spectrum (the filter's
// Chebyshev polynomials grow without limit beyond their interval): the solve
// restarts on [lmin, max(2 lmax, 1.5 x a fresh 120-step Lanczos estimate)], the
// third time on the rigorous bound of lmax_rigorous; batched solves share one
// interval and report the error.
void filtered_eig(const nm_pencil* P, double a, double b, int nev, double tol, const nm_eig_opts& o,
                  nm_eig_result** out, BatchSeat* seat, rocblas_handle blas) {
  nm_eig_opts oo = o;
  for (int attempt = 0;; ++attempt) {
    try {
      filtered_eig_once(P, a, b, nev, tol, oo, out, seat, blas);
      return;
    } catch (const FilterBlowUp& e) {
      if (seat || attempt >= 3) throw Error(NM_ENOCONV, e.what());
      double lo = 0, hi = 0;
      spectrum_bounds(P, 120, o.seed ^ 0x2545f491ull, (hipStream_t)o.stream, &lo, &hi);
      oo.lmin = std::min(e.lmin, lo - 1e-3 * (b - a));
      oo.lmax = std::max(2.0 * e.lmax, 1.5 * hi);
      // the last attempt takes the rigorous bound (when no self-gravitation term is attached)
      if (attempt == 2 && !P->selfgrav) oo.lmax = std::max(oo.lmax, lmax_rigorous(P, (hipStream_t)o.stream));
      if (o.verbose)
        fprintf(stderr, "[nmodes] filter blow-up with lambda_max %.6g: restarting on [%.6g, %.6g]\n", e.lmax, oo.lmin,
                oo.lmax);
    }
  }
}

static void filtered_eig_once(const nm_pencil* P, double a, double b, int nev, double tol, const nm_eig_opts& o,
                              nm_eig_result** out, BatchSeat* seat, rocblas_handle blas) {
  FilterBatcher* fb = seat ? seat->fb : nullptr;
  NM_REQUIRE(b > a && nev > 0 && tol > 0, NM_EINVAL, "need a < b, nev > 0, tol > 0");
  hipStream_t st = (hipStream_t)o.stream;
  Timer clock;
  const int64_t N = P->N, n = 3 * N;
  const int prec = o.precision;
  NM_REQUIRE(prec == 0 || prec == 1, NM_EINVAL, "precision must be 0 or 1");
  if (prec == 1) const_cast<nm_pencil*>(P)->ensure_fp32(st);
  int bs = solve_block_width(P, o, nev);
  check_block(n, bs);
  int Kmax = o.max_basis > 0 ? o.max_basis
                            : (int)std::min<int64_t>(n, std::max({6 * nev, nev + 16 * bs, 320}));
  Kmax = std::max(Kmax / bs, 2) * bs;
  Kmax = (int)std::min<int64_t>(Kmax, n / bs * bs);
  NM_REQUIRE(Kmax >= 2 * bs, NM_EINVAL, "problem too small for the block size");

  ApplyCfg cfg;
  KernelProf prof;
  cfg.prof = &prof;
  // default mass-solve bound: the residual floor it leaves is about half of it
  double mtol = o.minv_tol > 0 ? o.minv_tol : (prec ? 1e-7 : std::min(1e-7, std::max(1e-12, 0.3 * tol)));
  double ptol = o.kp_tol > 0 ? o.kp_tol : (prec ? 1e-7 : 1e-13);
  cfg.kM = cheb_steps(P->ref.m_lo, P->ref.m_hi, mtol);
  cfg.kP = cheb_steps(P->ref.p_lo, P->ref.p_hi, ptol);
  cfg.precision = prec;
  set_mass_passes(const_cast<nm_pencil*>(P), cfg, o.mass_passes, mtol, 0, st);
  Blas bl{blas ? blas : P->blas, st, {}};
  NM_BLAS(rocblas_set_stream(bl.h, st));
  NM_BLAS(rocblas_set_pointer_mode(bl.h, rocblas_pointer_mode_host));

  // ---------------- spectrum bounds (FP64 Lanczos in the M-inner product)
  double lmin = o.lmin, lmax = o.lmax;
  if (!(lmax > lmin)) {
    spectrum_bounds(P, 60, o.seed ^ 0x5bd1e995ull, st, &lmin, &lmax);
    lmin -= 1e-3 * (b - a);
  }
  NM_REQUIRE(lmax > b, NM_EINVAL, "window lies above the spectrum (b >= lambda_max)");

  // ---------------- filter
  // lower-side treatment (see choose_degree): explicit null factor, or,
  // by default, no damping below a when the pencil has fluid (its spectrum
  // below the window is the exactly degenerate Cowling null space) and
  // damping below a otherwise
  int mode = o.null_filter == 1 ? 2 : (o.null_filter == 0 ? 1 : (P->n_pres > 0 ? 0 : 1));
  if (o.null_filter == 2) mode = 0;
  if (o.null_filter == 3) mode = 3;
  NM_REQUIRE(o.null_filter >= -1 && o.null_filter <= 3, NM_EINVAL, "null_filter must be -1..3");
  const bool null = mode == 2;
  NM_REQUIRE(!(null && fb), NM_EINVAL, "batched solves do not take the null factor");
  const double l0 = 0.0, s0 = null ? b : 0.0;
  const int m = o.degree > 0 ? o.degree : choose_degree(a, b, lmin, lmax, o.guard, mode);
  std::vector<double> mu(m + 1);
  jackson_chebyshev(a, b, lmin, lmax, m, mu.data());
  const double c = 0.5 * (lmax + lmin), e = 0.5 * (lmax - lmin);
  const double tau = std::min(filter_value(mu, m, c, e, a, null, s0), filter_value(mu, m, c, e, b, null, s0));

  // ---------------- basis
  DBuf<double> V((size_t)n * Kmax), AV((size_t)n * Kmax);
  DBuf<double> W((size_t)n * bs), MW((size_t)n * bs), T2((size_t)n * bs), Cd((size_t)Kmax * bs),
      Gd((size_t)bs * bs);
  FilterWork<double> fw;
  FilterWork<float> fw32;
  DBuf<float> x32, y32;
  if (prec) {
    x32.alloc((size_t)n * bs);
    y32.alloc((size_t)n * bs);
  }
  std::vector<double> H((size_t)Kmax * Kmax, 0.0);  // Arnoldi coefficients of p(B), col-major
  double filter_time = 0.0, bytes = 0.0;
  int64_t bapps = 0;

  // FP64 operators of the pencil itself (Rayleigh-Ritz, residuals, M-inner products)
  ApplyCfg cfg64;
  cfg64.kM = cheb_steps(P->ref.m_lo, P->ref.m_hi, 1e-12);
  cfg64.kP = cheb_steps(P->ref.p_lo, P->ref.p_hi, 1e-13);
  cfg64.precision = 0;
  auto mprod = [&](const double* X, double* Y, int nc) { apply_op(P, NM_OP_M, nc, X, Y, cfg64, st); };
  // orthogonalise W (n x bs) against V[:, :K] (twice) and M-normalise by Cholesky QR (twice);
  // returns false on rank deficiency
  auto orthonormalise = [&](int K, double* Hcol, double* Rblk) -> bool {
    std::vector<double> Ch((size_t)std::max(K, 1) * bs);
    for (int pass = 0; pass < 2 && K > 0; ++pass) {
      mprod(W.p, MW.p, bs);
      bl.tn(n, K, bs, V.p, Kmax, MW.p, bs, Cd.p);
      bl.nn(n, K, bs, -1.0, V.p, Kmax, Cd.p, K, 1.0, W.p, bs);
      if (Hcol) {
        NM_HIP(hipMemcpyAsync(Ch.data(), Cd.p, 8 * (size_t)K * bs, hipMemcpyDeviceToHost, st));
        NM_HIP(hipStreamSynchronize(st));
        for (int v = 0; v < bs; ++v)
          for (int i = 0; i < K; ++i) Hcol[(size_t)i + (size_t)v * Kmax] += Ch[i + (size_t)v * K];
      }
    }
    std::vector<double> Rtot(bs * bs, 0.0);
    for (int i = 0; i < bs; ++i) Rtot[i + i * bs] = 1.0;
    for (int pass = 0; pass < 2; ++pass) {
      mprod(W.p, MW.p, bs);
      bl.tn(n, bs, bs, W.p, bs, MW.p, bs, Gd.p);
      std::vector<double> G(bs * bs), Ri;
      NM_HIP(hipMemcpyAsync(G.data(), Gd.p, 8 * bs * bs, hipMemcpyDeviceToHost, st));
      NM_HIP(hipStreamSynchronize(st));
      for (int i = 0; i < bs; ++i)
        for (int j = 0; j < i; ++j) G[i + j * bs] = G[j + i * bs] = 0.5 * (G[i + j * bs] + G[j + i * bs]);
      double gmax = 0;
      for (int i = 0; i < bs; ++i) gmax = std::max(gmax, G[i + i * bs]);
      bool ok;
      chol_upper(bs, G, ok);
      if (!ok) return false;
      double rmin = 1e300;
      for (int i = 0; i < bs; ++i) rmin = std::min(rmin, G[i + i * bs]);
      if (rmin * rmin < 1e-24 * gmax) return false;
      upper_inverse(bs, G, Ri);
      NM_HIP(hipMemcpyAsync(Gd.p, Ri.data(), 8 * bs * bs, hipMemcpyHostToDevice, st));
      bl.nn(n, bs, bs, 1.0, W.p, bs, Gd.p, bs, 0.0, T2.p, bs);
      std::swap(W.p, T2.p);
      // Rtot = R_pass * Rtot
      std::vector<double> Rn(bs * bs, 0.0);
      for (int i = 0; i < bs; ++i)
        for (int j = 0; j < bs; ++j) {
          double s = 0;
          for (int k = 0; k < bs; ++k) s += G[i + k * bs] * Rtot[k + j * bs];
          Rn[i + j * bs] = s;
        }
      Rtot = Rn;
    }
    if (Rblk) std::copy(Rtot.begin(), Rtot.end(), Rblk);
    return true;
  };
  auto put_block = [&](int K) {
    NM_HIP(hipMemcpy2DAsync(V.p + K, 8 * (size_t)Kmax, W.p, 8 * (size_t)bs, 8 * (size_t)bs, n,
                            hipMemcpyDeviceToDevice, st));
    apply_op(P, NM_OP_A, bs, W.p, MW.p, cfg64, st);
    NM_HIP(hipMemcpy2DAsync(AV.p + K, 8 * (size_t)Kmax, MW.p, 8 * (size_t)bs, 8 * (size_t)bs, n,
                            hipMemcpyDeviceToDevice, st));
  };

  // symmetric eigenproblem (col-major n x n, ascending values, vectors in columns):
  // cyclic Jacobi on the host for small orders, rocSOLVER dsyevd otherwise
  DBuf<rocblas_int> info(1);
  auto sym_eig = [&](int nn, std::vector<double>& A, std::vector<double>& wv, std::vector<double>& Sv) {
    if (nn <= 160) {
      jacobi_eig(nn, A, wv, &Sv);
      return;
    }
    DBuf<double> hd((size_t)nn * nn), wd(nn), ed(nn);
    NM_HIP(hipMemcpyAsync(hd.p, A.data(), 8 * (size_t)nn * nn, hipMemcpyHostToDevice, st));
    NM_BLAS(rocsolver_dsyevd(bl.h, rocblas_evect_original, rocblas_fill_upper, nn, hd.p, nn, wd.p, ed.p, info.p));
    wv.resize(nn);
    Sv.resize((size_t)nn * nn);
    NM_HIP(hipMemcpyAsync(wv.data(), wd.p, 8 * (size_t)nn, hipMemcpyDeviceToHost, st));
    NM_HIP(hipMemcpyAsync(Sv.data(), hd.p, 8 * (size_t)nn * nn, hipMemcpyDeviceToHost, st));
    NM_HIP(hipStreamSynchronize(st));
  };
  // convergence of the Ritz values of p(B): residual estimate <= mu_tol * max |Ritz value|;
  // an FP32 filter cannot take them much below 1e-6
  const double mu_tol = prec ? 1e-5 : 1e-8;

  uint64_t seed = o.seed;
  int64_t fresh = 0;
  auto random_block = [&]() {
    hipLaunchKernelGGL(k_randn, dim3(grid_for(n * bs)), dim3(256), 0, st, n, bs, bs, seed, fresh, W.p);
    fresh += bs;
  };
  random_block();
  NM_REQUIRE(orthonormalise(0, nullptr, nullptr), NM_ENOCONV, "start block is rank deficient");
  put_block(0);
  int K = bs;  // columns in V

  // results of the last Rayleigh-Ritz
  std::vector<double> th_sel, res_sel;
  std::vector<int> idx_sel;
  int last_count = -1;
  double prev_res_max = 0.0;
  bool converged = false;
  int Kc_last = 0;
  std::vector<double> Ysel;  // col-major Kc x nsel

  // Small problems are launch-bound (the filter is m (kM + ...) launches per
  // block): capture one filter application into a HIP graph on a private
  // stream, with fixed input and output buffers, and replay it for every
  // block.  NM_GRAPH=0/1 overrides the size rule.
  const char* genv = getenv("NM_GRAPH");
  const bool use_graph = !fb && (genv ? atoi(genv) != 0 : (double)n * bs <= 4.0e6);
  struct GraphState {
    hipStream_t gs = nullptr;
    hipGraphExec_t exec = nullptr;
    ~GraphState() {
      if (exec) (void)hipGraphExecDestroy(exec);
      if (gs) (void)hipStreamDestroy(gs);
    }
  } graph;
  DBuf<double> gin, gout;
  if (use_graph) {
    NM_HIP(hipStreamCreateWithFlags(&graph.gs, hipStreamNonBlocking));
    gin.alloc((size_t)n * bs);
    gout.alloc((size_t)n * bs);
  }

  for (int j = 0;; ++j) {
    const int Kj = K - bs;  // first column of the block to filter
    // ---- filter
    Timer ft;
    const double* vj = nullptr;
    int napp = m + (null ? 1 : 0);
    if (use_graph) {
      NM_HIP(hipMemcpy2DAsync(gin.p, 8 * (size_t)bs, V.p + Kj, 8 * (size_t)Kmax, 8 * (size_t)bs, n,
                              hipMemcpyDeviceToDevice, st));
      NM_HIP(hipStreamSynchronize(st));
      if (!graph.exec) {
        ApplyCfg gc = cfg;
        gc.prof = nullptr;  // no event records inside the graph
        if (prec == 0) {
          fw.ensure(P, bs);
          if (cfg.mixP) fw.ensure_mixed(P, bs);
        } else {
          fw32.ensure(P, bs);
        }
        hipGraph_t g = nullptr;
        NM_HIP(hipStreamBeginCapture(graph.gs, hipStreamCaptureModeThreadLocal));
        if (prec == 0) {
          filter_apply<double>(P, mu.data(), m, c, e, l0, s0, bs, gin.p, gout.p, gc, fw, graph.gs);
        } else {
          convert_f64_f32(n * bs, gin.p, x32.p, graph.gs);
          filter_apply<float>(P, mu.data(), m, c, e, l0, s0, bs, x32.p, y32.p, gc, fw32, graph.gs);
          convert_f32_f64(n * bs, y32.p, gout.p, graph.gs);
        }
        NM_HIP(hipStreamEndCapture(graph.gs, &g));
        const hipError_t ie = hipGraphInstantiate(&graph.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        NM_HIP(ie);
      }
      NM_HIP(hipGraphLaunch(graph.exec, graph.gs));
      NM_HIP(hipStreamSynchronize(graph.gs));
      NM_HIP(hipMemcpyAsync(W.p, gout.p, 8 * (size_t)n * bs, hipMemcpyDeviceToDevice, st));
    } else if (fb) {
      NM_HIP(hipMemcpy2DAsync(T2.p, 8 * (size_t)bs, V.p + Kj, 8 * (size_t)Kmax, 8 * (size_t)bs, n,
                              hipMemcpyDeviceToDevice, st));
      NM_HIP(hipStreamSynchronize(st));
      napp = fb->filter(T2.p, W.p, mu.data(), m, bs);
    } else if (prec == 0) {
      fw.ensure(P, bs);
      NM_HIP(hipMemcpy2DAsync(fw.x0.p, 8 * (size_t)bs, V.p + Kj, 8 * (size_t)Kmax, 8 * (size_t)bs, n,
                              hipMemcpyDeviceToDevice, st));
      vj = fw.x0.p;
      filter_apply<double>(P, mu.data(), m, c, e, l0, s0, bs, vj, W.p, cfg, fw, st);
    } else {
      fw32.ensure(P, bs);
      NM_HIP(hipMemcpy2DAsync(T2.p, 8 * (size_t)bs, V.p + Kj, 8 * (size_t)Kmax, 8 * (size_t)bs, n,
                              hipMemcpyDeviceToDevice, st));
      convert_f64_f32(n * bs, T2.p, x32.p, st);
      filter_apply<float>(P, mu.data(), m, c, e, l0, s0, bs, x32.p, y32.p, cfg, fw32, st);
      convert_f32_f64(n * bs, y32.p, W.p, st);
    }
    NM_HIP(hipStreamSynchronize(st));
    filter_time += ft.s();
    bapps += (int64_t)napp * bs;
    {
      // algorithmic bytes of one column B-application (matrices amortised over bs columns)
      const double s = prec ? 4.0 : 8.0;
      const double nnzb = (double)P->nnzb;
      double per = (nnzb * (9 * s + 4) + (cfg.kM - 1) * nnzb * (s + 4)) / bs + (4.0 * (cfg.kM - 1) + 4.0) * n * s;
      if (cfg.mixP) {
        // A (FP64 values, X, F), the first iterate (f, f32, y), FP32 steps (values and 4
        // streams), residuals (FP64 values; y, r in, r32, next iterate, and where kept the
        // FP64 residual and the sum) and the final sum with the filter update (5 streams)
        const int Pm = cfg.mixP;
        per = nnzb * (9 * 8.0 + 4) / bs + 16.0 * n + 16.0 * n + Pm * (cfg.mixK - 1.0) * (nnzb * 8.0 / bs + 16.0 * n);
        for (int q = 0; q + 1 < Pm; ++q)
          per += nnzb * 12.0 / bs + 20.0 * n + (q + 2 < Pm ? 8.0 * n : 0.0) +
                 (q >= 1 ? 8.0 * n + (q >= 2 ? 8.0 * n : 4.0 * n) : 0.0);
        per += (Pm >= 3 ? 12.0 : 8.0) * n + 40.0 * n;
      }
      bytes += per * napp * bs;
    }
    // ---- blow-up guard
    {
      std::vector<double> nr(bs);
      mprod(W.p, MW.p, bs);
      col_dots(n, bs, W.p, bs, MW.p, bs, Gd.p, st);
      d2h_sync(nr.data(), Gd.p, bs, st);
      for (double x : nr)
        if (!std::isfinite(x) || x > 1e30) throw FilterBlowUp(lmin, lmax);
    }
    if (K + bs > Kmax) break;
    // ---- orthogonalise, extend the basis
    std::vector<double> Rb(bs * bs);
    bool ok = orthonormalise(K, H.data() + (size_t)Kj * Kmax, Rb.data());
    if (ok) {
      for (int v = 0; v < bs; ++v)
        for (int i = 0; i < bs; ++i) H[(size_t)(K + i) + (size_t)(Kj + v) * Kmax] = Rb[i + v * bs];
    } else {
      // breakdown: the filtered space is (numerically) invariant; restart with fresh directions
      for (int tries = 0; tries < 3 && !ok; ++tries) {
        random_block();
        ok = orthonormalise(K, nullptr, nullptr);
      }
      NM_REQUIRE(ok, NM_ENOCONV, "block Lanczos breakdown could not be recovered");
    }
    put_block(K);
    K += bs;

    // ---- Ritz values of p(B) on the filtered part of the basis, their
    // residual estimates, and Rayleigh-Ritz with (A, M) restricted to the
    // span of the Ritz vectors of p(B) whose value is at least the filter's
    // window-edge level tau.  Restricting the Rayleigh-Ritz to that span keeps
    // out combinations of filtered-through directions far below the window
    // (the fluid null space) and above it, whose Rayleigh quotients can fall
    // inside the window without being eigenvalues.
    const int Kf = K - bs;  // columns whose images are in the basis
    if (Kf < bs && K + bs <= Kmax) continue;
    std::vector<double> w, S;
    {
      std::vector<double> Hs((size_t)Kf * Kf);
      for (int q = 0; q < Kf; ++q)
        for (int i = 0; i < Kf; ++i)
          Hs[i + (size_t)q * Kf] = 0.5 * (H[(size_t)i + (size_t)q * Kmax] + H[(size_t)q + (size_t)i * Kmax]);
      sym_eig(Kf, Hs, w, S);
    }
    bool mu_ok = true;
    std::vector<int> big;
    {
      double wmax = 0;
      for (double x : w) wmax = std::max(wmax, std::fabs(x));
      for (int i = 0; i < Kf; ++i) {
        if (w[i] < tau) continue;
        big.push_back(i);
        // residual estimate || H[K-bs:K, Kf-bs:Kf] s_i[Kf-bs:Kf] ||
        double r2 = 0;
        for (int p = 0; p < bs; ++p) {
          double sum = 0;
          for (int q = 0; q < bs; ++q)
            sum += H[(size_t)(Kf + p) + (size_t)(Kf - bs + q) * Kmax] * S[(size_t)(Kf - bs + q) + (size_t)i * Kf];
          r2 += sum * sum;
        }
        if (std::sqrt(r2) > mu_tol * wmax) mu_ok = false;
      }
    }
    const int nb = (int)big.size();
    std::vector<double> Yb((size_t)Kf * std::max(nb, 1));  // Kf x nb, col-major
    for (int q = 0; q < nb; ++q)
      std::copy(S.begin() + (size_t)big[q] * Kf, S.begin() + (size_t)(big[q] + 1) * Kf, Yb.begin() + (size_t)q * Kf);
    std::vector<double> th, Z;
    if (nb > 0) {
      // G = Yb^T (V_f^T A V_f) Yb on the device, then its eigenpairs
      DBuf<double> Ybd((size_t)Kf * nb), HAf((size_t)Kf * Kf), T1((size_t)Kf * nb), Gd2((size_t)nb * nb);
      NM_HIP(hipMemcpyAsync(Ybd.p, Yb.data(), 8 * Yb.size(), hipMemcpyHostToDevice, st));
      bl.tn(n, Kf, Kf, V.p, Kmax, AV.p, Kmax, HAf.p);
      const double one = 1.0, zero = 0.0;
      NM_BLAS(rocblas_dgemm(bl.h, rocblas_operation_none, rocblas_operation_none, Kf, nb, Kf, &one, HAf.p, Kf, Ybd.p,
                            Kf, &zero, T1.p, Kf));
      NM_BLAS(rocblas_dgemm(bl.h, rocblas_operation_transpose, rocblas_operation_none, nb, nb, Kf, &one, Ybd.p, Kf,
                            T1.p, Kf, &zero, Gd2.p, nb));
      std::vector<double> Gh((size_t)nb * nb);
      NM_HIP(hipMemcpyAsync(Gh.data(), Gd2.p, 8 * Gh.size(), hipMemcpyDeviceToHost, st));
      NM_HIP(hipStreamSynchronize(st));
      for (int i = 0; i < nb; ++i)
        for (int q = 0; q < i; ++q)
          Gh[i + (size_t)q * nb] = Gh[q + (size_t)i * nb] = 0.5 * (Gh[i + (size_t)q * nb] + Gh[q + (size_t)i * nb]);
      sym_eig(nb, Gh, th, Z);
    }
    idx_sel.clear();
    for (int i = 0; i < nb; ++i)
      if (th[i] >= a && th[i] <= b) idx_sel.push_back(i);
    const int ns = (int)idx_sel.size();
    th_sel.assign(ns, 0.0);
    res_sel.assign(ns, 0.0);
    // coefficients of the selected Ritz vectors in V_f: Yb Z[:, sel] (Kf x ns)
    std::vector<double> Ynew((size_t)Kf * std::max(ns, 0), 0.0);
    for (int q = 0; q < ns; ++q) {
      const double* zc = Z.data() + (size_t)idx_sel[q] * nb;
      double* yc = Ynew.data() + (size_t)q * Kf;
      for (int k = 0; k < nb; ++k) {
        const double zk = zc[k];
        const double* bc = Yb.data() + (size_t)k * Kf;
        for (int i = 0; i < Kf; ++i) yc[i] += zk * bc[i];
      }
    }
    bool res_ok = ns > 0;
    if (ns > 0) {
      DBuf<double> Yd((size_t)Kf * ns), X((size_t)n * ns), AX((size_t)n * ns), MX((size_t)n * ns), th_dev(ns),
          rn(ns), mn(ns);
      NM_HIP(hipMemcpyAsync(Yd.p, Ynew.data(), 8 * Ynew.size(), hipMemcpyHostToDevice, st));
      bl.nn(n, Kf, ns, 1.0, V.p, Kmax, Yd.p, Kf, 0.0, X.p, ns);
      bl.nn(n, Kf, ns, 1.0, AV.p, Kmax, Yd.p, Kf, 0.0, AX.p, ns);
      mprod(X.p, MX.p, ns);
      for (int i = 0; i < ns; ++i) th_sel[i] = th[idx_sel[i]];
      NM_HIP(hipMemcpyAsync(th_dev.p, th_sel.data(), 8 * ns, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_sub_scaled_cols, dim3(grid_for(n * ns)), dim3(256), 0, st, n, ns, AX.p, MX.p, th_dev.p,
                         AX.p);
      col_dots(n, ns, AX.p, ns, AX.p, ns, rn.p, st);
      col_dots(n, ns, MX.p, ns, MX.p, ns, mn.p, st);
      std::vector<double> r2(ns), m2(ns);
      d2h_sync(r2.data(), rn.p, ns, st);
      d2h_sync(m2.data(), mn.p, ns, st);
      for (int i = 0; i < ns; ++i) {
        res_sel[i] = std::sqrt(r2[i]) / (std::fabs(th_sel[i]) * std::sqrt(m2[i]));
        if (i < nev && !(res_sel[i] <= tol)) res_ok = false;  // the pairs returned: the nev lowest
      }
    }
    if (o.verbose)
      fprintf(stderr, "[nmodes] block %d basis %d window-pairs %d resid-max %.2e big-mu %d mu-ok %d t=%.2fs\n", j, K,
              ns, ns ? *std::max_element(res_sel.begin(), res_sel.end()) : 0.0, nb, (int)mu_ok, clock.s());
    bool stable = ns == last_count;
    last_count = ns;
    Kc_last = Kf;
    Ysel = std::move(Ynew);
    // Rounding in the filter (FP64: eps64 times the degree; FP32: eps32) puts
    // noise into every spectral component, which the residual weighs by
    // lambda_j / lambda: the window residuals stall at a floor.  Stop when
    // they are below tol or have stopped improving (refined below).
    // With refinement available, residuals within 10 tol are handed to it as soon as p(B) has
    // converged (the last block before the floor only shaves the residual there; at 100 tol the
    // remaining error is partly unconverged Krylov directions, which the refinement cannot fix).
    const int nret = std::min(ns, nev);
    const double res_max = nret ? *std::max_element(res_sel.begin(), res_sel.begin() + nret) : 0.0;
    const bool stalled = ns > 0 && prev_res_max > 0 && res_max > 0.5 * prev_res_max;
    const bool refinable = o.refine >= 0 && ns > 0 && res_max <= 10.0 * tol;
    prev_res_max = res_max;
    if ((res_ok || stalled || refinable) && stable && mu_ok) {
      converged = true;
      break;
    }
    if (K + bs > Kmax) break;
  }

  // this solve submits no more filter blocks
  if (seat) seat->leave();
  fb = nullptr;

  // ---------------- FP64 refinement of the window pairs
  // The refined set is the window Ritz vectors plus the Ritz vectors of the
  // full basis just above the window, (b, b (1 + guard)], and below it (not
  // the null cluster): the window vectors' remaining error lies mostly along
  // those (the filter damps them least, the low-pass q below amplifies the
  // ones under the window), so the Rayleigh-Ritz of the refined set needs
  // them.  Every vector of the set is refined; the noisy basis itself is not
  // used (it holds a second, noisy copy of each window eigenvector, and
  // Rayleigh-Ritz over both mixes them).
  DBuf<double> Xref;  // refined Ritz vectors (internal order), [n][xref_ld], window vectors first
  int xref_ld = 0;
  int refine_passes = 0, kq = 0;
  int64_t refine_bapps = 0;
  Timer rclock;
  // largest residual among the pairs returned (the nev lowest of the window)
  auto max_res = [&]() {
    const size_t k = std::min(res_sel.size(), (size_t)nev);
    return k ? *std::max_element(res_sel.begin(), res_sel.begin() + k) : 0.0;
  };
  if (o.refine >= 0 && !th_sel.empty() && max_res() > tol) {
    const int npass = o.refine > 0 ? o.refine : 3;
    const int ns0 = (int)th_sel.size();
    const int Kf = Kc_last;
    const double gd = o.guard > 0 ? o.guard : 1.0;
    // upper end of the band refined with the window: b (1 + guard), or for slices b + guard (b - a)
    const double bband = mode == 3 ? b + gd * (b - a) : b * (1.0 + gd);
    // FP32 basis: null factor in the refinement (see the low-pass below)
    const bool nullf = prec == 1;
    // window vectors (restricted Rayleigh-Ritz) and band vectors (full Rayleigh-Ritz over V_f)
    std::vector<double> Yband;
    int nband = 0;
    {
      DBuf<double> HAf((size_t)Kf * Kf);
      bl.tn(n, Kf, Kf, V.p, Kmax, AV.p, Kmax, HAf.p);
      std::vector<double> h((size_t)Kf * Kf), thf, Zf;
      NM_HIP(hipMemcpyAsync(h.data(), HAf.p, 8 * h.size(), hipMemcpyDeviceToHost, st));
      NM_HIP(hipStreamSynchronize(st));
      for (int q = 0; q < Kf; ++q)
        for (int i = 0; i < q; ++i) h[i + (size_t)q * Kf] = h[q + (size_t)i * Kf] = 0.5 * (h[i + (size_t)q * Kf] + h[q + (size_t)i * Kf]);
      sym_eig(Kf, h, thf, Zf);
      for (int i = 0; i < Kf; ++i)
        if ((thf[i] > b && thf[i] <= bband) || (thf[i] < a && std::fabs(thf[i]) > 1e-6 * b)) {
          Yband.insert(Yband.end(), Zf.begin() + (size_t)i * Kf, Zf.begin() + (size_t)(i + 1) * Kf);
          ++nband;
        }
    }
    int nsel = ns0;
    const int qt0 = ns0 + nband;
    DBuf<double> Xw((size_t)n * qt0);  // [window | band], row-major [n][qt]
    {
      std::vector<double> Ycat(Ysel.begin(), Ysel.begin() + (size_t)Kf * ns0);
      Ycat.insert(Ycat.end(), Yband.begin(), Yband.end());
      DBuf<double> Yd((size_t)Kf * qt0);
      NM_HIP(hipMemcpyAsync(Yd.p, Ycat.data(), 8 * Ycat.size(), hipMemcpyHostToDevice, st));
      bl.nn(n, Kf, qt0, 1.0, V.p, Kmax, Yd.p, Kf, 0.0, Xw.p, qt0);
      NM_HIP(hipStreamSynchronize(st));
    }
    int qt = qt0;
    // low-pass q(t) = T_k((c_q - t) / e_q) / T_k((c_q - b) / e_q) with [c_q -+ e_q] = [lc, lmax]:
    // positive and decreasing below lc, 1 at b, |q| <= d on [lc, lmax].  The rounding noise of
    // the basis is spread over the spectrum and weighed by lambda_j / lambda in the residual; to
    // lower the Lanczos floor r0 by f = tol / (10 r0), components above lc = lmax f^(2/3) are
    // damped to d = f / 3 (with a Weyl-law density the weighted noise left below lc scales as
    // (lc / lmax)^(3/2)).  q grows below b, by up to (6 / f)^0.41 at 0: harmless for the
    // FP64-level null-space content of an FP64 basis, not for an FP32 one, whose refined vectors
    // are therefore (B / b) q(B) X -- the factor removes the exactly degenerate null space (the
    // fluid kernel of the Cowling operator).  With the large degree an FP32 floor asks for, q
    // falls fast enough above b to absorb the factor's growth lambda / b; with the small degree
    // of an FP64 floor it would not, which is why FP64 goes without it.
    const double r0 = max_res();
    const double f = std::min(0.5, std::max(1e-12, tol / (10.0 * r0)));
    const double lc = std::min(std::max(b * (1.0 + gd), lmax * std::pow(f, 2.0 / 3.0)), 0.5 * (b + lmax));
    const double dq = f / 3.0;
    const double tb = 1.0 + 2.0 * (lc - b) / (lmax - lc);
    kq = std::max(2, (int)std::ceil(std::acosh(1.0 / dq) / std::acosh(tb)));
    std::vector<double> muq(kq + 1, 0.0);
    muq[kq] = ((kq & 1) ? -1.0 : 1.0) / std::cosh(kq * std::acosh(tb));
    const double cq = 0.5 * (lmax + lc), eq = 0.5 * (lmax - lc);
    ApplyCfg cfgq = cfg64;
    cfgq.kM = cheb_steps(P->ref.m_lo, P->ref.m_hi, std::min(1e-7, std::max(1e-12, 0.3 * tol)));
    fw.ensure(P, bs);
    double prev = r0;
    for (int pass = 0; pass < npass; ++pass) {
      const int q = qt;
      // Y = q(B) X (FP32 basis: (B / b) q(B) X), bs columns at a time
      DBuf<double> Yq((size_t)n * q), MY((size_t)n * q), AY((size_t)n * q);
      for (int j0 = 0; j0 < q; j0 += bs) {
        const int nc = std::min(bs, q - j0);
        NM_HIP(hipMemcpy2DAsync(T2.p, 8 * (size_t)nc, Xw.p + j0, 8 * (size_t)q, 8 * (size_t)nc, n,
                                hipMemcpyDeviceToDevice, st));
        filter_apply<double>(P, muq.data(), kq, cq, eq, 0.0, nullf ? b : 0.0, nc, T2.p, W.p, cfgq, fw, st);
        NM_HIP(hipMemcpy2DAsync(Yq.p + j0, 8 * (size_t)q, W.p, 8 * (size_t)nc, 8 * (size_t)nc, n,
                                hipMemcpyDeviceToDevice, st));
        if (o.verbose) {
          // progress of long refinements (an FP32 basis needs a high degree on many vectors)
          NM_HIP(hipStreamSynchronize(st));
          fprintf(stderr, "[nmodes] refine pass %d: columns %d..%d of %d filtered (degree %d) t=%.2fs\n", pass, j0,
                  j0 + nc, q, kq, rclock.s());
        }
      }
      refine_bapps += (int64_t)(kq + (nullf ? 1 : 0)) * q;
      // drop columns that the null factor has (numerically) annihilated, then
      // M-orthonormalise by Cholesky QR (twice)
      {
        DBuf<double> nd(q);
        mprod(Yq.p, MY.p, q);
        col_dots(n, q, Yq.p, q, MY.p, q, nd.p, st);
        std::vector<double> nrm(q);
        d2h_sync(nrm.data(), nd.p, q, st);
        const double mx = *std::max_element(nrm.begin(), nrm.end());
        std::vector<int> live;
        for (int k = 0; k < q; ++k)
          if (nrm[k] > 1e-20 * mx) live.push_back(k);
        if ((int)live.size() < q) {
          const int ql = (int)live.size();
          for (int k = 0; k < ql; ++k)
            NM_HIP(hipMemcpy2DAsync(MY.p + k, 8 * (size_t)ql, Yq.p + live[k], 8 * (size_t)q, 8, n,
                                    hipMemcpyDeviceToDevice, st));
          NM_HIP(hipMemcpyAsync(Yq.p, MY.p, 8 * (size_t)n * ql, hipMemcpyDeviceToDevice, st));
          qt = ql;
        }
      }
      // M-orthonormalise (twice): Cholesky QR, or, when the Gram matrix is numerically singular
      // (the refined vectors can be nearly dependent: q is far from flat across the window when
      // its degree is high), an eigendecomposition of the scaled Gram matrix that drops the
      // directions below 1e-12 of the largest
      bool ok = true;
      for (int it = 0; it < 2 && ok; ++it) {
        const int qc = qt;
        DBuf<double> Gq((size_t)qc * qc);
        mprod(Yq.p, MY.p, qc);
        bl.tn(n, qc, qc, Yq.p, qc, MY.p, qc, Gq.p);
        std::vector<double> G((size_t)qc * qc), gw, GU;
        NM_HIP(hipMemcpyAsync(G.data(), Gq.p, 8 * G.size(), hipMemcpyDeviceToHost, st));
        NM_HIP(hipStreamSynchronize(st));
        {
          std::vector<double> Gc(G), Ri;
          for (int i = 0; i < qc; ++i)
            for (int k = 0; k < i; ++k)
              Gc[i + (size_t)k * qc] = Gc[k + (size_t)i * qc] = 0.5 * (Gc[i + (size_t)k * qc] + Gc[k + (size_t)i * qc]);
          bool cok = true;
          chol_upper(qc, Gc, cok);
          if (cok) {
            upper_inverse(qc, Gc, Ri);
            NM_HIP(hipMemcpyAsync(Gq.p, Ri.data(), 8 * Ri.size(), hipMemcpyHostToDevice, st));
            bl.nn(n, qc, qc, 1.0, Yq.p, qc, Gq.p, qc, 0.0, MY.p, qc);
            std::swap(Yq.p, MY.p);
            continue;
          }
        }
        std::vector<double> dsc(qc);
        for (int i = 0; i < qc; ++i) dsc[i] = G[i + (size_t)i * qc] > 0 ? 1.0 / std::sqrt(G[i + (size_t)i * qc]) : 0.0;
        for (int k = 0; k < qc; ++k)
          for (int i = 0; i < qc; ++i) {
            const double g = 0.5 * (G[i + (size_t)k * qc] + G[k + (size_t)i * qc]);
            G[i + (size_t)k * qc] = dsc[i] * g * dsc[k];
          }
        sym_eig(qc, G, gw, GU);
        const double wmax = gw.empty() ? 0.0 : gw.back();
        std::vector<int> kept;
        for (int k = 0; k < qc; ++k)
          if (gw[k] > 1e-12 * wmax) kept.push_back(k);
        const int r = (int)kept.size();
        if (r == 0) {
          ok = false;
          break;
        }
        std::vector<double> Cm((size_t)qc * r);
        for (int c2 = 0; c2 < r; ++c2) {
          const int k = kept[c2];
          const double sc = 1.0 / std::sqrt(gw[k]);
          for (int i = 0; i < qc; ++i) Cm[i + (size_t)c2 * qc] = dsc[i] * GU[i + (size_t)k * qc] * sc;
        }
        DBuf<double> Cd2((size_t)qc * r);
        NM_HIP(hipMemcpyAsync(Cd2.p, Cm.data(), 8 * Cm.size(), hipMemcpyHostToDevice, st));
        bl.nn(n, qc, r, 1.0, Yq.p, qc, Cd2.p, qc, 0.0, MY.p, r);
        NM_HIP(hipMemcpyAsync(Yq.p, MY.p, 8 * (size_t)n * r, hipMemcpyDeviceToDevice, st));
        qt = r;
      }
      const int q2 = qt;
      if (!ok) break;  // the refined set is (numerically) rank deficient
      apply_op(P, NM_OP_A, q2, Yq.p, AY.p, cfg64, st);
      // Rayleigh-Ritz with (A, M) on span(Y)
      DBuf<double> Hd((size_t)q2 * q2);
      bl.tn(n, q2, q2, Yq.p, q2, AY.p, q2, Hd.p);
      std::vector<double> Ht((size_t)q2 * q2), tht, Zt;
      NM_HIP(hipMemcpyAsync(Ht.data(), Hd.p, 8 * Ht.size(), hipMemcpyDeviceToHost, st));
      NM_HIP(hipStreamSynchronize(st));
      for (int i = 0; i < q2; ++i)
        for (int k = 0; k < i; ++k) Ht[i + (size_t)k * q2] = Ht[k + (size_t)i * q2] = 0.5 * (Ht[i + (size_t)k * q2] + Ht[k + (size_t)i * q2]);
      sym_eig(q2, Ht, tht, Zt);
      std::vector<int> cand, keep;
      for (int i = 0; i < q2; ++i) {
        if (tht[i] >= a && tht[i] <= b) cand.push_back(i);
        if ((tht[i] > b && tht[i] <= bband) || (tht[i] < a && std::fabs(tht[i]) > 1e-6 * b))
          keep.push_back(i);
      }
      const int nc = (int)cand.size();
      if (nc == 0) break;
      // all window candidates and the band vectors of this Rayleigh-Ritz (next pass's set)
      std::vector<int> all(cand);
      all.insert(all.end(), keep.begin(), keep.end());
      const int na = (int)all.size();
      std::vector<double> za((size_t)q2 * na), thc(nc);
      for (int k = 0; k < na; ++k)
        std::copy(Zt.begin() + (size_t)all[k] * q2, Zt.begin() + (size_t)(all[k] + 1) * q2, za.begin() + (size_t)k * q2);
      for (int k = 0; k < nc; ++k) thc[k] = tht[cand[k]];
      DBuf<double> zad((size_t)q2 * na), Xc((size_t)n * na), AXc((size_t)n * nc), MXc((size_t)n * nc), thd(nc),
          rn(nc), mn(nc);
      NM_HIP(hipMemcpyAsync(zad.p, za.data(), 8 * za.size(), hipMemcpyHostToDevice, st));
      NM_HIP(hipMemcpyAsync(thd.p, thc.data(), 8 * nc, hipMemcpyHostToDevice, st));
      bl.nn(n, q2, na, 1.0, Yq.p, q2, zad.p, q2, 0.0, Xc.p, na);
      bl.nn(n, q2, nc, 1.0, AY.p, q2, zad.p, q2, 0.0, AXc.p, nc);
      DBuf<double> Xwin((size_t)n * nc);
      NM_HIP(hipMemcpy2DAsync(Xwin.p, 8 * (size_t)nc, Xc.p, 8 * (size_t)na, 8 * (size_t)nc, n,
                              hipMemcpyDeviceToDevice, st));
      mprod(Xwin.p, MXc.p, nc);
      hipLaunchKernelGGL(k_sub_scaled_cols, dim3(grid_for(n * nc)), dim3(256), 0, st, n, nc, AXc.p, MXc.p, thd.p,
                         AXc.p);
      col_dots(n, nc, AXc.p, nc, AXc.p, nc, rn.p, st);
      col_dots(n, nc, MXc.p, nc, MXc.p, nc, mn.p, st);
      std::vector<double> r2(nc), m2(nc), rc(nc);
      d2h_sync(r2.data(), rn.p, nc, st);
      d2h_sync(m2.data(), mn.p, nc, st);
      for (int k = 0; k < nc; ++k) rc[k] = std::sqrt(r2[k]) / (std::fabs(thc[k]) * std::sqrt(m2[k]));
      // keep the ns0 window candidates of smallest residual, ascending
      std::vector<int> ord(nc);
      std::iota(ord.begin(), ord.end(), 0);
      std::sort(ord.begin(), ord.end(), [&](int x, int y) { return rc[x] < rc[y]; });
      ord.resize(std::min(nc, ns0));
      std::sort(ord.begin(), ord.end());
      nsel = (int)ord.size();
      th_sel.assign(nsel, 0.0);
      res_sel.assign(nsel, 0.0);
      bool all_ok = true;
      // next set: [selected window vectors | band vectors]
      const int nb2 = (int)keep.size();
      DBuf<double> Xn((size_t)n * (nsel + nb2));
      for (int k = 0; k < nsel; ++k) {
        th_sel[k] = thc[ord[k]];
        res_sel[k] = rc[ord[k]];
        all_ok = all_ok && (k >= nev || res_sel[k] <= tol);
        NM_HIP(hipMemcpy2DAsync(Xn.p + k, 8 * (size_t)(nsel + nb2), Xc.p + ord[k], 8 * (size_t)na, 8, n,
                                hipMemcpyDeviceToDevice, st));
      }
      if (nb2)
        NM_HIP(hipMemcpy2DAsync(Xn.p + nsel, 8 * (size_t)(nsel + nb2), Xc.p + nc, 8 * (size_t)na, 8 * (size_t)nb2, n,
                                hipMemcpyDeviceToDevice, st));
      Xw = std::move(Xn);
      qt = nsel + nb2;
      ++refine_passes;
      if (o.verbose)
        fprintf(stderr, "[nmodes] refine pass %d degree %d pairs %d (+%d above) resid-max %.2e t=%.2fs\n", pass, kq,
                nsel, nb2, max_res(), clock.s());
      if (all_ok || max_res() > 0.5 * prev) break;
      prev = max_res();
    }
    if (refine_passes > 0) {
      Xref = std::move(Xw);  // window vectors first
      xref_ld = qt;
    }
  }
  const double refine_seconds = refine_passes > 0 ? rclock.s() : 0.0;

  // ---------------- result: the min(nev, count) smallest pairs in the window
  const int ns = (int)th_sel.size();
  const int cnt = std::min(nev, ns);
  int nconv = 0;
  for (int i = 0; i < cnt; ++i) nconv += res_sel[i] <= tol;
  nm_eig_result* r = new nm_eig_result();
  memset(r, 0, sizeof(*r));
  r->count = cnt;
  r->n = n;
  r->lambda = (double*)std::malloc(8 * std::max(cnt, 1));
  r->resid = (double*)std::malloc(8 * std::max(cnt, 1));
  for (int i = 0; i < cnt; ++i) {
    r->lambda[i] = th_sel[i];
    r->resid[i] = res_sel[i];
  }
  if (cnt > 0) {
    DBuf<double> sg(cnt);
    NM_HIP(hipMalloc((void**)&r->X, 8 * (size_t)n * cnt));
    // Ritz vectors in the internal node order, then to the canonical order
    DBuf<double> Xi((size_t)n * cnt);
    if (refine_passes > 0) {
      NM_HIP(hipMemcpy2DAsync(Xi.p, 8 * (size_t)cnt, Xref.p, 8 * (size_t)xref_ld, 8 * (size_t)cnt, n,
                              hipMemcpyDeviceToDevice, st));
    } else {
      DBuf<double> Yd((size_t)Kc_last * cnt);
      NM_HIP(hipMemcpyAsync(Yd.p, Ysel.data(), 8 * (size_t)Kc_last * cnt, hipMemcpyHostToDevice, st));
      bl.nn(n, Kc_last, cnt, 1.0, V.p, Kmax, Yd.p, Kc_last, 0.0, Xi.p, cnt);
    }
    permute_rows(N, 3 * cnt, Xi.p, r->X, P->perm.p, 8, st);
    hipLaunchKernelGGL(k_col_sign, dim3(cnt), dim3(256), 0, st, n, cnt, r->X, sg.p);
    hipLaunchKernelGGL(k_scale_cols, dim3(grid_for(n * cnt)), dim3(256), 0, st, n, cnt, sg.p, r->X);
  }
  NM_HIP(hipStreamSynchronize(st));
  r->degree = m;
  r->kM = cfg.kM;
  r->kP = cfg.kP;
  r->block = bs;
  r->basis = K;
  r->bapps = bapps;
  r->lmin = lmin;
  r->lmax = lmax;
  r->bytes = bytes;
  r->filter_seconds = filter_time;
  prof.harvest();
  r->hot_launches = prof.launches;
  r->hot_samples = prof.samples;
  r->hot_ms = prof.samples ? prof.ms / prof.samples : 0.0;
  {
    // a middle step of the FP64 mass solve, or of an FP32 pass of the mixed one
    const double sz = (prec || cfg.mixP) ? 4.0 : 8.0;
    r->hot_bytes = (double)P->nnzb * (4.0 + sz) + 4.0 * (P->N + 1) + sz * P->N + 4.0 * n * bs * sz;
  }
  r->mass_passes = cfg.mixP;
  r->mass_pass_steps = cfg.mixP ? cfg.mixK : cfg.kM;
  r->hot_kernel = mass_kernel_kind(P, bs, prec == 1 || cfg.mixP > 0);
  r->refine_passes = refine_passes;
  r->refine_degree = kq;
  r->refine_seconds = refine_seconds;
  r->refine_bapps = refine_bapps;
  r->seconds = clock.s();
  *out = r;
  if (!converged || nconv < cnt) throw Error(NM_PARTIAL, "solve did not converge all pairs in the window");
}

}  // namespace nm
