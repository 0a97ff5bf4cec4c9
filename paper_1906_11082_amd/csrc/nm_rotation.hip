// Rotating modes by projection (Sec. 7 of the paper): with the M-orthonormal
// non-rotating eigenvectors X_e (A X_e = M X_e Lambda_e, eq. "linearpb") the
// linearised Coriolis QEP projects to
//   [[0, L], [L, 2iS]] [y; w y] = w [[L, 0], [0, I]] [y; w y],  S = X_e^T R X_e
// (eq. "sublinear0").  Scaling by diag(L^{-1/2}, I) gives the Hermitian
// standard problem [[0, L^{1/2}], [L^{1/2}, 2iS]] v = w v, solved on the
// device; modes u = X_e y are normalised by eq. "orthonormalcond".
#include <rocsolver/rocsolver.h>

#include <chrono>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>

#include <cstdio>
#include <cstdlib>

#include "nm_internal.h"

namespace nm {
namespace {

__device__ __forceinline__ int64_t gtid() { return nm_xcd_block() * blockDim.x + threadIdx.x; }

__global__ void k_interleave(int64_t rows, int nc, const double* __restrict__ re, const double* __restrict__ im,
                             double* __restrict__ out) {
  int64_t g = gtid();
  if (g >= rows * nc) return;
  out[2 * g] = re[g];
  out[2 * g + 1] = im[g];
}

__global__ void k_deinterleave(int64_t rows, int nc, const double* __restrict__ in, double* __restrict__ re,
                               int ldr, double* __restrict__ im, int ldi) {
  int64_t g = gtid();
  if (g >= rows * nc) return;
  const int64_t r = g / nc;
  const int v = (int)(g - r * nc);
  re[r * ldr + v] = in[2 * g];
  im[r * ldi + v] = in[2 * g + 1];
}

// QEP residual of modes u = ur + i ui (columns v and k + v of [n][2k] blocks MX, RX, AX):
// r = w^2 M u - 2 i w R u - A u, written as Re r (column v) and Im r (column k + v) of Rr
__global__ void k_qep_resid(int64_t rows, int k, const double* __restrict__ om, const double* __restrict__ MX,
                            const double* __restrict__ RX, const double* __restrict__ AX, double* __restrict__ Rr) {
  int64_t g = gtid();
  if (g >= rows * k) return;
  const int64_t r = g / k;
  const int v = (int)(g - r * k);
  const double w = om[v];
  const int64_t a = r * 2 * k + v, b = a + k;
  Rr[a] = w * w * MX[a] + 2.0 * w * RX[b] - AX[a];
  Rr[b] = w * w * MX[b] - 2.0 * w * RX[a] - AX[b];
}

// phase of each column: entry of largest modulus made real positive
__global__ void k_phase(int64_t rows, int nc, double* U) {
  int v = blockIdx.x;
  __shared__ double bm[256], br[256], bi[256];
  double best = -1, pr = 1, pi = 0;
  for (int64_t r = threadIdx.x; r < rows; r += blockDim.x) {
    double x = U[2 * (r * nc + v)], y = U[2 * (r * nc + v) + 1];
    double m = x * x + y * y;
    if (m > best) { best = m; pr = x; pi = y; }
  }
  bm[threadIdx.x] = best; br[threadIdx.x] = pr; bi[threadIdx.x] = pi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o && bm[threadIdx.x + o] > bm[threadIdx.x]) {
      bm[threadIdx.x] = bm[threadIdx.x + o]; br[threadIdx.x] = br[threadIdx.x + o]; bi[threadIdx.x] = bi[threadIdx.x + o];
    }
    __syncthreads();
  }
  double a = br[0], b = bi[0], m = sqrt(a * a + b * b);
  double cr = m > 0 ? a / m : 1.0, ci = m > 0 ? -b / m : 0.0;  // conj(phase)
  for (int64_t r = threadIdx.x; r < rows; r += blockDim.x) {
    double x = U[2 * (r * nc + v)], y = U[2 * (r * nc + v) + 1];
    U[2 * (r * nc + v)] = x * cr - y * ci;
    U[2 * (r * nc + v) + 1] = x * ci + y * cr;
  }
}

}  // namespace

// QEP residuals ||w^2 M u - 2 i w R u - A u|| / (w^2 ||M u||) of the modes of r (canonical order)
void rotation_residuals(const nm_pencil* P, nm_rot_result* r, hipStream_t st) {
  const int k = r->count;
  std::free(r->resid);
  r->resid = (double*)std::calloc(std::max(k, 1), sizeof(double));
  if (k == 0) return;
  const int64_t n = r->n;
  DBuf<double> X2((size_t)n * 2 * k), MX((size_t)n * 2 * k), RX((size_t)n * 2 * k), AX((size_t)n * 2 * k), om(k),
      d1(2 * k), d2(2 * k);
  hipLaunchKernelGGL(k_deinterleave, dim3(grid_for(n * k)), dim3(256), 0, st, n, k, r->U, X2.p, 2 * k, X2.p + k,
                     2 * k);
  ApplyCfg cfg;
  cfg.kP = cheb_steps(P->ref.p_lo, P->ref.p_hi, 1e-13);
  cfg.kM = cheb_steps(P->ref.m_lo, P->ref.m_hi, 1e-12);
  api_apply(P, NM_OP_M, 2 * k, X2.p, MX.p, cfg, st);
  api_apply(P, NM_OP_R, 2 * k, X2.p, RX.p, cfg, st);
  api_apply(P, NM_OP_A, 2 * k, X2.p, AX.p, cfg, st);
  NM_HIP(hipMemcpyAsync(om.p, r->omega, 8 * k, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_qep_resid, dim3(grid_for(n * k)), dim3(256), 0, st, n, k, om.p, MX.p, RX.p, AX.p, X2.p);
  col_dots(n, 2 * k, X2.p, 2 * k, X2.p, 2 * k, d1.p, st);
  col_dots(n, 2 * k, MX.p, 2 * k, MX.p, 2 * k, d2.p, st);
  std::vector<double> h1(2 * k), h2(2 * k);
  NM_HIP(hipMemcpyAsync(h1.data(), d1.p, 16 * k, hipMemcpyDeviceToHost, st));
  NM_HIP(hipMemcpyAsync(h2.data(), d2.p, 16 * k, hipMemcpyDeviceToHost, st));
  NM_HIP(hipStreamSynchronize(st));
  for (int v = 0; v < k; ++v) {
    const double w = r->omega[v];
    r->resid[v] = std::sqrt(h1[v] + h1[k + v]) / (w * w * std::sqrt(h2[v] + h2[k + v]));
  }
}

namespace {

// The projection of eq. "sublinear0" on an M-orthonormal basis X with
// X^T A X = diag(lambda).  With lambda > 0 (eigenpairs of the pencil) the
// mode's coefficients are the upper half of the Hermitian eigenvector over
// sqrt(lambda); with zero_ok (a Rayleigh-Ritz basis that may hold rigid
// motions or null-space directions, lambda >= 0) they are the lower half
// over omega, which needs no division by sqrt(lambda).
void project_core(const nm_pencil* P, const nm_eig_result* B, double a, double b, hipStream_t st,
                  nm_rot_result** out, bool zero_ok) {
  auto t0 = std::chrono::steady_clock::now();
  NM_REQUIRE(B && B->count > 0 && B->X, NM_EINVAL, "empty basis");
  const int m = B->count;
  const int64_t n = B->n;
  NM_REQUIRE(n == 3 * P->N, NM_EINVAL, "basis does not belong to this pencil");
  for (int i = 0; i < m; ++i)
    NM_REQUIRE(zero_ok ? B->lambda[i] >= 0 : B->lambda[i] > 0, NM_EINVAL, "projection needs positive eigenvalues");
  NM_BLAS(rocblas_set_stream(P->blas, st));
  NM_BLAS(rocblas_set_pointer_mode(P->blas, rocblas_pointer_mode_host));
  DBuf<double> RX((size_t)n * m), Sd((size_t)m * m);
  ApplyCfg cfg;
  api_apply(P, NM_OP_R, m, B->X, RX.p, cfg, st);
  // S (col-major m x m) = X^T R X
  DBuf<double> ws;
  gemm_tn(n, m, m, B->X, m, RX.p, m, Sd.p, ws, st);
  std::vector<double> S((size_t)m * m);
  NM_HIP(hipMemcpyAsync(S.data(), Sd.p, 8 * S.size(), hipMemcpyDeviceToHost, st));
  NM_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < i; ++j) {
      double s = 0.5 * (S[i + (size_t)j * m] - S[j + (size_t)i * m]);
      S[i + (size_t)j * m] = s;
      S[j + (size_t)i * m] = -s;
    }
  for (int i = 0; i < m; ++i) S[i + (size_t)i * m] = 0.0;
  const int n2 = 2 * m;
  std::vector<std::complex<double>> H((size_t)n2 * n2, 0.0);
  for (int i = 0; i < m; ++i) {
    double r = std::sqrt(B->lambda[i]);
    H[i + (size_t)(m + i) * n2] = r;
    H[(m + i) + (size_t)i * n2] = r;
    for (int j = 0; j < m; ++j) H[(m + i) + (size_t)(m + j) * n2] = std::complex<double>(0.0, 2.0 * S[i + (size_t)j * m]);
  }
  DBuf<rocblas_double_complex> Hd((size_t)n2 * n2);
  DBuf<double> wd(n2), ed(n2);
  DBuf<rocblas_int> info(1);
  NM_HIP(hipMemcpyAsync(Hd.p, H.data(), 16 * H.size(), hipMemcpyHostToDevice, st));
  NM_BLAS(rocsolver_zheevd(P->blas, rocblas_evect_original, rocblas_fill_upper, n2, Hd.p, n2, wd.p, ed.p, info.p));
  std::vector<double> w(n2);
  NM_HIP(hipMemcpyAsync(w.data(), wd.p, 8 * n2, hipMemcpyDeviceToHost, st));
  NM_HIP(hipMemcpyAsync(H.data(), Hd.p, 16 * H.size(), hipMemcpyDeviceToHost, st));
  NM_HIP(hipStreamSynchronize(st));
  std::vector<int> keep;
  for (int i = 0; i < n2; ++i)
    if (w[i] > 0 && w[i] * w[i] >= a && w[i] * w[i] <= b) keep.push_back(i);
  const int k = (int)keep.size();
  nm_rot_result* r = (nm_rot_result*)calloc(1, sizeof(nm_rot_result));
  r->count = k;
  r->n = n;
  r->omega = (double*)malloc(8 * std::max(k, 1));
  if (k > 0) {
    // y = v[:m] / sqrt(lambda) (or v[m:] / w), normalised by y^H y - (i/w) y^H S y = 1
    std::vector<double> Yr((size_t)m * k), Yi((size_t)m * k);
    for (int q = 0; q < k; ++q) {
      const int col = keep[q];
      const double om = w[col];
      r->omega[q] = om;
      std::vector<std::complex<double>> y(m);
      for (int i = 0; i < m; ++i)
        y[i] = zero_ok ? H[(m + i) + (size_t)col * n2] / om : H[i + (size_t)col * n2] / std::sqrt(B->lambda[i]);
      std::complex<double> yy = 0, ysy = 0;
      for (int i = 0; i < m; ++i) {
        yy += std::conj(y[i]) * y[i];
        std::complex<double> sy = 0;
        for (int j = 0; j < m; ++j) sy += S[i + (size_t)j * m] * y[j];
        ysy += std::conj(y[i]) * sy;
      }
      double nrm = std::real(yy - std::complex<double>(0.0, 1.0 / om) * ysy);
      double sc = 1.0 / std::sqrt(nrm);
      for (int i = 0; i < m; ++i) {
        Yr[i + (size_t)q * m] = y[i].real() * sc;
        Yi[i + (size_t)q * m] = y[i].imag() * sc;
      }
    }
    DBuf<double> Yrd(Yr.size()), Yid(Yi.size()), Ur((size_t)n * k), Ui((size_t)n * k);
    NM_HIP(hipMemcpyAsync(Yrd.p, Yr.data(), 8 * Yr.size(), hipMemcpyHostToDevice, st));
    NM_HIP(hipMemcpyAsync(Yid.p, Yi.data(), 8 * Yi.size(), hipMemcpyHostToDevice, st));
    // U (row-major [n][k]) = X Y : U^T = Y^T X^T
    gemm_nn(n, m, k, 1.0, B->X, m, Yrd.p, m, 0.0, Ur.p, k, st);
    gemm_nn(n, m, k, 1.0, B->X, m, Yid.p, m, 0.0, Ui.p, k, st);
    NM_HIP(hipMalloc((void**)&r->U, 16 * (size_t)n * k));
    hipLaunchKernelGGL(k_interleave, dim3(grid_for(n * k)), dim3(256), 0, st, n, k, Ur.p, Ui.p, r->U);
    hipLaunchKernelGGL(k_phase, dim3(k), dim3(256), 0, st, n, k, r->U);
    NM_HIP(hipStreamSynchronize(st));
  }
  rotation_residuals(P, r, st);
  r->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = r;
}

}  // namespace

void project_rotation(const nm_pencil* P, const nm_eig_result* B, double a, double b, hipStream_t st,
                      nm_rot_result** out) {
  project_core(P, B, a, b, st, out, false);
}

namespace {

// Jackson-damped Chebyshev interpolation on [lmin, lmax] (degree d) of the
// regularised resolvent g(l) = (l - s) / ((l - s)^2 + q^2): coefficients mu[0..d]
void resolvent_series(double s, double q, double lmin, double lmax, int d, double* mu) {
  const double c = 0.5 * (lmax + lmin), e = 0.5 * (lmax - lmin);
  const int nn = 4 * d + 8;
  std::vector<double> th(nn), fv(nn);
  for (int i = 0; i < nn; ++i) {
    th[i] = M_PI * (i + 0.5) / nn;
    const double x = c + e * std::cos(th[i]) - s;
    fv[i] = x / (x * x + q * q);
  }
  const double tj = M_PI / (d + 2);
  for (int k = 0; k <= d; ++k) {
    double acc = 0.0;
    for (int i = 0; i < nn; ++i) acc += fv[i] * std::cos(k * th[i]);
    acc *= 2.0 / nn;
    if (k == 0) acc *= 0.5;
    const double jac = ((1.0 - (double)k / (d + 2)) * std::sin(tj) * std::cos(k * tj) +
                        std::cos(tj) * std::sin(k * tj) / (d + 2)) / std::sin(tj);
    mu[k] = acc * jac;
  }
}

// symmetric eigenproblem of a column-major n x n host matrix (ascending): rocSOLVER on the device
void sym_eig_dev(rocblas_handle h, int nn, std::vector<double>& A, std::vector<double>& w, hipStream_t st) {
  DBuf<double> ad((size_t)nn * nn), wd(nn), ed(nn);
  DBuf<rocblas_int> info(1);
  NM_HIP(hipMemcpyAsync(ad.p, A.data(), 8 * A.size(), hipMemcpyHostToDevice, st));
  NM_BLAS(rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, nn, ad.p, nn, wd.p, ed.p, info.p));
  w.resize(nn);
  NM_HIP(hipMemcpyAsync(w.data(), wd.p, 8 * nn, hipMemcpyDeviceToHost, st));
  NM_HIP(hipMemcpyAsync(A.data(), ad.p, 8 * A.size(), hipMemcpyDeviceToHost, st));
  NM_HIP(hipStreamSynchronize(st));
}

}  // namespace

// Refinement of projected rotating modes toward the exact QEP (Sec. 7, eq.
// "simplequad"; the text after eq. "sublinear0" notes that the projection's
// accuracy improves by solving the QEP exactly).  The projection is a
// Rayleigh-Ritz on span(X_e); here the span grows: each pass takes every
// mode's QEP residual r = w^2 M u - 2 i w R u - A u and adds the directions
// g_w(B) M^{-1} Re r and g_w(B) M^{-1} Im r, g_w the Jackson-damped Chebyshev
// series of the regularised resolvent (l - w^2) / ((l - w^2)^2 + (w^2/4)^2)
// (the first-order correction of u along the eigenvector of eigenvalue l is
// its residual component over w^2 - l), M-orthonormalised against the span.
// The enlarged span V is rotated to the eigenvectors of K = V^T A V (dropping
// directions with K-eigenvalue below 1e-10 of the largest), and the projected
// problem of eq. "sublinear0" is solved on it (project_rotation with
// Lambda_e = those eigenvalues).  Rigid motions and the fluid null space of A,
// which the window basis leaves out, enter through the corrections.
void refine_rotation(const nm_pencil* P, const nm_eig_result* B, const nm_rot_result* R0, double a, double b,
                     int iters, int degree, double tol, hipStream_t st, nm_rot_result** out) {
  auto t0 = std::chrono::steady_clock::now();
  NM_REQUIRE(B && B->count > 0 && B->X && R0, NM_EINVAL, "refinement needs the window basis and its projection");
  NM_REQUIRE(B->n == 3 * P->N && R0->n == B->n, NM_EINVAL, "basis does not belong to this pencil");
  NM_REQUIRE(B->lmax > B->lmin, NM_EINVAL, "the basis carries no spectrum bounds");
  NM_REQUIRE(iters >= 0 && tol > 0, NM_EINVAL, "need iters >= 0 and tol > 0");
  const int64_t n = B->n, N = P->N;
  const int m0 = B->count;
  const bool verbose = std::getenv("NM_REFINE_VERBOSE") != nullptr;
  const int d = degree > 0 ? degree
                           : std::min(2000, std::max(100, (int)std::ceil(20.0 * std::sqrt(B->lmax / b))));
  NM_BLAS(rocblas_set_stream(P->blas, st));
  NM_BLAS(rocblas_set_pointer_mode(P->blas, rocblas_pointer_mode_host));
  rocblas_handle h = P->blas;
  ApplyCfg cfg;
  cfg.kM = cheb_steps(P->ref.m_lo, P->ref.m_hi, 1e-12);
  cfg.kP = cheb_steps(P->ref.p_lo, P->ref.p_hi, 1e-13);
  DBuf<double> ws;  // row-chunk partials of the block products
  // basis V and A V (canonical order, row-major [n][ld]); capacity for every pass's corrections
  const int kmax = R0->count;
  const int ld = m0 + iters * 2 * std::max(kmax, 1) + 2 * std::max(kmax, 1);
  DBuf<double> V((size_t)n * ld), AV((size_t)n * ld);
  NM_HIP(hipMemcpy2DAsync(V.p, 8 * (size_t)ld, B->X, 8 * (size_t)m0, 8 * (size_t)m0, n, hipMemcpyDeviceToDevice, st));
  {
    DBuf<double> tmp((size_t)n * m0);
    api_apply(P, NM_OP_A, m0, B->X, tmp.p, cfg, st);
    NM_HIP(hipMemcpy2DAsync(AV.p, 8 * (size_t)ld, tmp.p, 8 * (size_t)m0, 8 * (size_t)m0, n, hipMemcpyDeviceToDevice,
                            st));
  }
  int m = m0;
  nm_rot_result* cur = nullptr;  // owned once refined
  const nm_rot_result* src = R0;
  int done_iters = 0;
  for (int it = 0; it < iters; ++it) {
    const int k = src->count;
    if (k == 0) break;
    double rmax = 0.0;
    for (int v = 0; v < k; ++v) rmax = std::max(rmax, src->resid ? src->resid[v] : 1.0);
    if (rmax <= tol) break;
    NM_REQUIRE(m + 2 * k <= ld, NM_EINVAL, "rotation refinement: basis capacity exceeded");
    // residual blocks [Re r | Im r]
    DBuf<double> X2((size_t)n * 2 * k), MX((size_t)n * 2 * k), RX((size_t)n * 2 * k), AX((size_t)n * 2 * k),
        om(k);
    hipLaunchKernelGGL(k_deinterleave, dim3(grid_for(n * k)), dim3(256), 0, st, n, k, src->U, X2.p, 2 * k,
                       X2.p + k, 2 * k);
    api_apply(P, NM_OP_M, 2 * k, X2.p, MX.p, cfg, st);
    api_apply(P, NM_OP_R, 2 * k, X2.p, RX.p, cfg, st);
    api_apply(P, NM_OP_A, 2 * k, X2.p, AX.p, cfg, st);
    NM_HIP(hipMemcpyAsync(om.p, src->omega, 8 * k, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_qep_resid, dim3(grid_for(n * k)), dim3(256), 0, st, n, k, om.p, MX.p, RX.p, AX.p, X2.p);
    // corrections G = g_w(B) M^{-1} r, in column blocks of at most 32 (internal node order for the filter)
    api_apply(P, NM_OP_MINV, 2 * k, X2.p, MX.p, cfg, st);  // MX now holds M^{-1} r
    const int nc = 2 * k;
    const double c = 0.5 * (B->lmax + B->lmin), e = 0.5 * (B->lmax - B->lmin);
    std::vector<std::vector<double>> mus(k, std::vector<double>(d + 1));
    for (int v = 0; v < k; ++v) {
      const double s2 = src->omega[v] * src->omega[v];
      resolvent_series(s2, 0.25 * s2, B->lmin, B->lmax, d, mus[v].data());
    }
    {
      FilterWork<double> fw;
      const int bs = 32;
      DBuf<double> xi((size_t)N * 3 * bs), yi((size_t)N * 3 * bs), xc((size_t)n * bs);
      for (int j0 = 0; j0 < nc; j0 += bs) {
        const int q = std::min(bs, nc - j0);
        std::vector<double> mc((size_t)(d + 1) * q);
        for (int kk = 0; kk <= d; ++kk)
          for (int jj = 0; jj < q; ++jj) mc[(size_t)kk * q + jj] = mus[(j0 + jj) % k][kk];
        NM_HIP(hipMemcpy2DAsync(xc.p, 8 * (size_t)q, MX.p + j0, 8 * (size_t)nc, 8 * (size_t)q, n,
                                hipMemcpyDeviceToDevice, st));
        permute_rows(N, 3 * q, xc.p, xi.p, P->iperm.p, 8, st);
        filter_apply_cols<double>(P, mc.data(), d, c, e, q, xi.p, yi.p, cfg, fw, st);
        permute_rows(N, 3 * q, yi.p, xc.p, P->perm.p, 8, st);
        NM_HIP(hipMemcpy2DAsync(AX.p + j0, 8 * (size_t)nc, xc.p, 8 * (size_t)q, 8 * (size_t)q, n,
                                hipMemcpyDeviceToDevice, st));
      }
    }
    double* G = AX.p;  // [n][nc] corrections
    // orthogonalise against V (M-inner product, twice): G -= V (V^T M G)
    DBuf<double> Cd((size_t)m * nc);
    for (int pass = 0; pass < 2; ++pass) {
      api_apply(P, NM_OP_M, nc, G, RX.p, cfg, st);
      gemm_tn(n, m, nc, V.p, ld, RX.p, nc, Cd.p, ws, st);
      gemm_nn(n, m, nc, -1.0, V.p, ld, Cd.p, m, 1.0, G, nc, st);
    }
    // M-orthonormalise G: eigenvectors of its (scaled) Gram matrix, dropping directions below 1e-10
    api_apply(P, NM_OP_M, nc, G, RX.p, cfg, st);
    DBuf<double> Gd((size_t)nc * nc);
    gemm_tn(n, nc, nc, G, nc, RX.p, nc, Gd.p, ws, st);
    std::vector<double> Gh((size_t)nc * nc), gw;
    NM_HIP(hipMemcpyAsync(Gh.data(), Gd.p, 8 * Gh.size(), hipMemcpyDeviceToHost, st));
    NM_HIP(hipStreamSynchronize(st));
    std::vector<double> dsc(nc);
    for (int i = 0; i < nc; ++i) dsc[i] = Gh[i + (size_t)i * nc] > 0 ? 1.0 / std::sqrt(Gh[i + (size_t)i * nc]) : 0.0;
    {
      // symmetrised and scaled to unit diagonal, into a fresh array (in place,
      // the second of each pair would read an already scaled partner)
      std::vector<double> Gs((size_t)nc * nc);
      for (int q = 0; q < nc; ++q)
        for (int i = 0; i < nc; ++i)
          Gs[i + (size_t)q * nc] = dsc[i] * 0.5 * (Gh[i + (size_t)q * nc] + Gh[q + (size_t)i * nc]) * dsc[q];
      Gh.swap(Gs);
    }
    sym_eig_dev(h, nc, Gh, gw, st);
    const double gmax = gw.empty() ? 0.0 : gw.back();
    std::vector<int> keep;
    for (int i = 0; i < nc; ++i)
      if (gw[i] > 1e-10 * gmax) keep.push_back(i);
    const int r = (int)keep.size();
    if (verbose)
      fprintf(stderr, "[nmodes] refine pass %d: %d modes, max resid %.3e, corrections %d of %d kept (Gram %.3e .. %.3e)\n",
              it, k, rmax, r, nc, gw.empty() ? 0.0 : gw.front(), gmax);
    if (r == 0) break;
    std::vector<double> Cm((size_t)nc * r);
    for (int c2 = 0; c2 < r; ++c2)
      for (int i = 0; i < nc; ++i)
        Cm[i + (size_t)c2 * nc] = dsc[i] * Gh[i + (size_t)keep[c2] * nc] / std::sqrt(gw[keep[c2]]);
    DBuf<double> Cmd((size_t)nc * r), Gn((size_t)n * r);
    NM_HIP(hipMemcpyAsync(Cmd.p, Cm.data(), 8 * Cm.size(), hipMemcpyHostToDevice, st));
    gemm_nn(n, nc, r, 1.0, G, nc, Cmd.p, nc, 0.0, Gn.p, r, st);
    NM_HIP(hipMemcpy2DAsync(V.p + m, 8 * (size_t)ld, Gn.p, 8 * (size_t)r, 8 * (size_t)r, n, hipMemcpyDeviceToDevice,
                            st));
    api_apply(P, NM_OP_A, r, Gn.p, MX.p, cfg, st);
    NM_HIP(hipMemcpy2DAsync(AV.p + m, 8 * (size_t)ld, MX.p, 8 * (size_t)r, 8 * (size_t)r, n, hipMemcpyDeviceToDevice,
                            st));
    m += r;
    // Rayleigh-Ritz: eigenvectors of K = V^T A V, then the projected problem on them
    DBuf<double> Kd((size_t)m * m);
    gemm_tn(n, m, m, V.p, ld, AV.p, ld, Kd.p, ws, st);
    std::vector<double> Kh((size_t)m * m), kw;
    NM_HIP(hipMemcpyAsync(Kh.data(), Kd.p, 8 * Kh.size(), hipMemcpyDeviceToHost, st));
    NM_HIP(hipStreamSynchronize(st));
    for (int q = 0; q < m; ++q)
      for (int i = 0; i < q; ++i) Kh[i + (size_t)q * m] = Kh[q + (size_t)i * m] = 0.5 * (Kh[i + (size_t)q * m] + Kh[q + (size_t)i * m]);
    sym_eig_dev(h, m, Kh, kw, st);
    // every direction of the enlarged span is kept, rigid motions and null
    // directions (K-eigenvalue ~ 0) included -- dropping them loses the
    // coupling the refinement is for; directions of clearly negative K (the
    // gravitational terms make A indefinite on a few) have no real frequency
    // and are left out
    const double kmx = kw.empty() ? 0.0 : kw.back();
    std::vector<int> kk;
    for (int i = 0; i < m; ++i)
      if (kw[i] >= -1e-10 * kmx) kk.push_back(i);
    const int mk = (int)kk.size();
    std::vector<double> Qk((size_t)m * mk), lam(mk);
    for (int q = 0; q < mk; ++q) {
      lam[q] = std::max(0.0, kw[kk[q]]);
      std::copy(Kh.begin() + (size_t)kk[q] * m, Kh.begin() + (size_t)(kk[q] + 1) * m, Qk.begin() + (size_t)q * m);
    }
    DBuf<double> Qd((size_t)m * mk), W((size_t)n * mk);
    NM_HIP(hipMemcpyAsync(Qd.p, Qk.data(), 8 * Qk.size(), hipMemcpyHostToDevice, st));
    gemm_nn(n, m, mk, 1.0, V.p, ld, Qd.p, m, 0.0, W.p, mk, st);
    nm_eig_result tmp;
    std::memset(&tmp, 0, sizeof(tmp));
    tmp.count = mk;
    tmp.n = n;
    tmp.lambda = lam.data();
    tmp.X = W.p;
    nm_rot_result* rn = nullptr;
    project_core(P, &tmp, a, b, st, &rn, true);
    // a pass is kept only if every mode it returns has a residual below the
    // previous pass's largest: Rayleigh-Ritz for the QEP has no min-max
    // principle, and on the enlarged span it can return spurious window
    // values with large residuals (measured on a small fluid planet); the
    // refinement then stops at its best pass
    double rn_max = 0.0;
    for (int v = 0; v < rn->count; ++v) rn_max = std::max(rn_max, rn->resid[v]);
    if (verbose)
      fprintf(stderr, "[nmodes] refine pass %d: basis %d (K %.3e .. %.3e, %d kept), %d modes, max resid %.3e\n", it,
              m, kw.empty() ? 0.0 : kw.front(), kmx, mk, rn->count, rn_max);
    if (rn->count == 0 || !(rn_max < rmax)) {
      nm_rot_result_free(rn);
      break;
    }
    if (cur) nm_rot_result_free(cur);
    cur = rn;
    src = cur;
    ++done_iters;
  }
  if (!cur) {
    // nothing to refine: a copy of the projection
    cur = (nm_rot_result*)std::calloc(1, sizeof(nm_rot_result));
    cur->count = R0->count;
    cur->n = n;
    cur->omega = (double*)std::malloc(8 * std::max(R0->count, 1));
    std::copy(R0->omega, R0->omega + R0->count, cur->omega);
    if (R0->count) {
      NM_HIP(hipMalloc((void**)&cur->U, 16 * (size_t)n * R0->count));
      NM_HIP(hipMemcpyAsync(cur->U, R0->U, 16 * (size_t)n * R0->count, hipMemcpyDeviceToDevice, st));
    }
    rotation_residuals(P, cur, st);
  }
  cur->iters = done_iters;
  cur->basis = m;
  cur->degree = d;
  cur->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = cur;
}

}  // namespace nm
