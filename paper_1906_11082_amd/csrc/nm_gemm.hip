// Dense block products of the Lanczos basis on the FP64 matrix cores.
//
// The basis V and its images are row-major [n][ld] with n in the millions
// and at most a few thousand columns, and the blocks they meet are narrow,
// so both products are tall and skinny:
//   gemm_tn: C = A^T B          (K x q, col-major; a reduction over the n rows),
//   gemm_nn: D = alpha A C + beta D   (n x q row-major; a reduction over K).
// They carry the Gram-Schmidt projections against the basis, the Cholesky
// Gram matrices and the Rayleigh-Ritz matrices of the filtered Lanczos
// (Sec. 6.2).  Each wavefront owns TM x TN output tiles of 16 x 16 and feeds
// v_mfma_f64_16x16x4f64 four rows (tn) or four basis columns (nn) per step.
// gemm_tn splits the rows into chunks whose partial products a second kernel
// sums in chunk order, so the result does not depend on scheduling.
#include "nm_internal.h"

namespace nm {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// Operand layout of v_mfma_f64_16x16x4f64 for lane l of the wavefront:
// A[i][k] with i = l % 16, k = l / 16; B[k][j] with j = l % 16, k = l / 16;
// the 16 x 16 result D[i][j] in four registers v: i = l / 16 + 4 v, j = l % 16
// (measured with single-entry operands on gfx950).
__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// part[chunk][k][j] = sum over the chunk's rows r of A[r][k] B[r][j], for the
// wavefront's k in [k0, k0 + 16 TM) and j in [j0, j0 + 16 TN)
template <int TM, int TN>
__global__ __launch_bounds__(64) void k_gemm_tn(int64_t n, int K, int q, const double* __restrict__ A, int lda,
                                                const double* __restrict__ B, int ldb, int64_t rows_per_chunk,
                                                double* __restrict__ part) {
  const int lane = threadIdx.x, li = lane & 15, lk = lane >> 4;
  const int64_t chunk = blockIdx.x;
  const int k0 = blockIdx.y * 16 * TM, j0 = blockIdx.z * 16 * TN;
  const int64_t r0 = chunk * rows_per_chunk, r1 = min(n, r0 + rows_per_chunk);
  d4 acc[TM][TN];
#pragma unroll
  for (int t = 0; t < TM; ++t)
#pragma unroll
    for (int u = 0; u < TN; ++u) acc[t][u] = d4{0.0, 0.0, 0.0, 0.0};
  for (int64_t r = r0; r < r1; r += 4) {
    const int64_t row = r + lk;
    const bool rin = row < r1;
    double a[TM], b[TN];
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const int k = k0 + 16 * t + li;
      a[t] = rin && k < K ? A[row * lda + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < TN; ++u) {
      const int j = j0 + 16 * u + li;
      b[u] = rin && j < q ? B[row * ldb + j] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < TM; ++t)
#pragma unroll
      for (int u = 0; u < TN; ++u) acc[t][u] = mfma_f64(a[t], b[u], acc[t][u]);
  }
  double* P = part + (size_t)chunk * K * q;
#pragma unroll
  for (int t = 0; t < TM; ++t)
#pragma unroll
    for (int u = 0; u < TN; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = k0 + 16 * t + lk + 4 * v, j = j0 + 16 * u + li;
        if (k < K && j < q) P[(size_t)k * q + j] = acc[t][u][v];
      }
}

// C[k + j K] = sum over chunks c (in order) of part[c][k][j]
__global__ void k_gemm_tn_sum(int K, int q, int nchunks, const double* __restrict__ part, double* __restrict__ C) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)K * q) return;
  const int k = (int)(i / q), j = (int)(i - (int64_t)k * q);
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += part[(size_t)c * K * q + i];
  C[k + (size_t)j * K] = s;
}

// D[r][j] = alpha sum_k A[r][k] C[k + j ldc] + beta D[r][j] (D not read when
// beta is 0).  A workgroup of 4 wavefronts owns 4 x 16 TM rows and the
// column block [j0, j0 + 16 TN); C is staged in LDS 64 basis columns at a time.
template <int TM, int TN>
__global__ __launch_bounds__(256) void k_gemm_nn(int64_t n, int K, int q, double alpha, const double* __restrict__ A,
                                                 int lda, const double* __restrict__ C, int ldc, double beta,
                                                 double* __restrict__ D, int ldd) {
  constexpr int KC = 64, JW = 16 * TN;
  __shared__ double sC[KC][JW];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int64_t rw = ((int64_t)blockIdx.x * 4 + wave) * 16 * TM;
  const int j0 = blockIdx.y * JW;
  d4 acc[TM][TN];
#pragma unroll
  for (int t = 0; t < TM; ++t)
#pragma unroll
    for (int u = 0; u < TN; ++u) acc[t][u] = d4{0.0, 0.0, 0.0, 0.0};
  for (int kc = 0; kc < K; kc += KC) {
    __syncthreads();
    for (int i = threadIdx.x; i < KC * JW; i += blockDim.x) {
      const int kk = i % KC, jj = i / KC;
      const int k = kc + kk, j = j0 + jj;
      sC[kk][jj] = k < K && j < q ? C[k + (size_t)j * ldc] : 0.0;
    }
    __syncthreads();
    const int kend = min(KC, K - kc);
    for (int ks = 0; ks < kend; ks += 4) {
      const int k = kc + ks + lk;
      double a[TM], b[TN];
#pragma unroll
      for (int t = 0; t < TM; ++t) {
        const int64_t row = rw + 16 * t + li;
        a[t] = row < n && k < K ? A[row * lda + k] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < TN; ++u) b[u] = sC[ks + lk][16 * u + li];
#pragma unroll
      for (int t = 0; t < TM; ++t)
#pragma unroll
        for (int u = 0; u < TN; ++u) acc[t][u] = mfma_f64(a[t], b[u], acc[t][u]);
    }
  }
#pragma unroll
  for (int t = 0; t < TM; ++t)
#pragma unroll
    for (int u = 0; u < TN; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = rw + 16 * t + lk + 4 * v;
        const int j = j0 + 16 * u + li;
        if (row < n && j < q) {
          double x = alpha * acc[t][u][v];
          if (beta != 0.0) x += beta * D[row * ldd + j];
          D[row * ldd + j] = x;
        }
      }
}

inline int col_tiles(int q) { return q <= 16 ? 1 : (q <= 32 ? 2 : 4); }

}  // namespace

void gemm_tn(int64_t n, int K, int q, const double* A, int lda, const double* B, int ldb, double* C, DBuf<double>& ws,
             hipStream_t st) {
  NM_REQUIRE(n >= 0 && K >= 0 && q >= 0 && lda >= K && ldb >= q, NM_EINVAL, "gemm_tn: bad sizes");
  if (K == 0 || q == 0) return;
  if (n == 0) {
    NM_HIP(hipMemsetAsync(C, 0, (size_t)K * q * sizeof(double), st));
    return;
  }
  constexpr int TM = 4;
  const int tn = col_tiles(q);
  const int kb = (K + 16 * TM - 1) / (16 * TM), jb = (q + 16 * tn - 1) / (16 * tn);
  // enough row chunks for ~4096 wavefronts, at least 256 rows each
  int64_t nchunks = std::max<int64_t>(1, (4096 + (int64_t)kb * jb - 1) / ((int64_t)kb * jb));
  nchunks = std::min<int64_t>(nchunks, std::max<int64_t>(1, n / 256));
  int64_t rpc = (n + nchunks - 1) / nchunks;
  rpc = (rpc + 3) / 4 * 4;
  nchunks = (n + rpc - 1) / rpc;
  const size_t need = (size_t)nchunks * K * q;
  if (ws.n < need) ws.alloc(need);
  const dim3 grid((unsigned)nchunks, (unsigned)kb, (unsigned)jb);
  if (tn == 1)
    hipLaunchKernelGGL((k_gemm_tn<TM, 1>), grid, dim3(64), 0, st, n, K, q, A, lda, B, ldb, rpc, ws.p);
  else if (tn == 2)
    hipLaunchKernelGGL((k_gemm_tn<TM, 2>), grid, dim3(64), 0, st, n, K, q, A, lda, B, ldb, rpc, ws.p);
  else
    hipLaunchKernelGGL((k_gemm_tn<TM, 4>), grid, dim3(64), 0, st, n, K, q, A, lda, B, ldb, rpc, ws.p);
  const int64_t outs = (int64_t)K * q;
  hipLaunchKernelGGL(k_gemm_tn_sum, dim3((unsigned)((outs + 255) / 256)), dim3(256), 0, st, K, q, (int)nchunks,
                     ws.p, C);
  NM_HIP(hipGetLastError());
}

void gemm_nn(int64_t n, int K, int q, double alpha, const double* A, int lda, const double* C, int ldc, double beta,
             double* D, int ldd, hipStream_t st) {
  NM_REQUIRE(n >= 0 && K >= 0 && q >= 0 && lda >= K && ldc >= K && ldd >= q, NM_EINVAL, "gemm_nn: bad sizes");
  NM_REQUIRE(n == 0 || q == 0 || (const void*)A != (const void*)D, NM_EINVAL, "gemm_nn: A and D must differ");
  if (n == 0 || q == 0) return;
  constexpr int TM = 4;
  const int tn = col_tiles(q);
  const int64_t rb = (n + 4 * 16 * TM - 1) / (4 * 16 * TM);
  const int jb = (q + 16 * tn - 1) / (16 * tn);
  NM_REQUIRE(rb < (int64_t)INT32_MAX, NM_EINVAL, "gemm_nn: too many rows");
  const dim3 grid((unsigned)rb, (unsigned)jb);
  if (tn == 1)
    hipLaunchKernelGGL((k_gemm_nn<TM, 1>), grid, dim3(256), 0, st, n, K, q, alpha, A, lda, C, ldc, beta, D, ldd);
  else if (tn == 2)
    hipLaunchKernelGGL((k_gemm_nn<TM, 2>), grid, dim3(256), 0, st, n, K, q, alpha, A, lda, C, ldc, beta, D, ldd);
  else
    hipLaunchKernelGGL((k_gemm_nn<TM, 4>), grid, dim3(256), 0, st, n, K, q, alpha, A, lda, C, ldc, beta, D, ldd);
  NM_HIP(hipGetLastError());
}

}  // namespace nm
