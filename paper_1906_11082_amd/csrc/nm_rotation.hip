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

void project_rotation(const nm_pencil* P, const nm_eig_result* B, double a, double b, hipStream_t st,
                      nm_rot_result** out) {
  auto t0 = std::chrono::steady_clock::now();
  NM_REQUIRE(B && B->count > 0 && B->X, NM_EINVAL, "empty basis");
  const int m = B->count;
  const int64_t n = B->n;
  NM_REQUIRE(n == 3 * P->N, NM_EINVAL, "basis does not belong to this pencil");
  for (int i = 0; i < m; ++i) NM_REQUIRE(B->lambda[i] > 0, NM_EINVAL, "projection needs positive eigenvalues");
  NM_BLAS(rocblas_set_stream(P->blas, st));
  NM_BLAS(rocblas_set_pointer_mode(P->blas, rocblas_pointer_mode_host));
  DBuf<double> RX((size_t)n * m), Sd((size_t)m * m);
  ApplyCfg cfg;
  api_apply(P, NM_OP_R, m, B->X, RX.p, cfg, st);
  const double one = 1.0, zero = 0.0;
  // S (col-major m x m) = X^T R X
  NM_BLAS(rocblas_dgemm(P->blas, rocblas_operation_none, rocblas_operation_transpose, m, m, (rocblas_int)n, &one,
                        B->X, m, RX.p, m, &zero, Sd.p, m));
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
    // y = v[:m] / sqrt(lambda), normalised by y^H y - (i/w) y^H S y = 1
    std::vector<double> Yr((size_t)m * k), Yi((size_t)m * k);
    for (int q = 0; q < k; ++q) {
      const int col = keep[q];
      const double om = w[col];
      r->omega[q] = om;
      std::vector<std::complex<double>> y(m);
      for (int i = 0; i < m; ++i) y[i] = H[i + (size_t)col * n2] / std::sqrt(B->lambda[i]);
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
    NM_BLAS(rocblas_dgemm(P->blas, rocblas_operation_transpose, rocblas_operation_none, k, (rocblas_int)n, m, &one,
                          Yrd.p, m, B->X, m, &zero, Ur.p, k));
    NM_BLAS(rocblas_dgemm(P->blas, rocblas_operation_transpose, rocblas_operation_none, k, (rocblas_int)n, m, &one,
                          Yid.p, m, B->X, m, &zero, Ui.p, k));
    NM_HIP(hipMalloc((void**)&r->U, 16 * (size_t)n * k));
    hipLaunchKernelGGL(k_interleave, dim3(grid_for(n * k)), dim3(256), 0, st, n, k, Ur.p, Ui.p, r->U);
    hipLaunchKernelGGL(k_phase, dim3(k), dim3(256), 0, st, n, k, r->U);
    NM_HIP(hipStreamSynchronize(st));
  }
  r->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = r;
}

}  // namespace nm
