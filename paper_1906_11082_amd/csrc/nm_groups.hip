// Row groups of the node graph for the grouped mass-solve kernel.
//
// Rows (displacement nodes, in the internal Hilbert-curve order) are grouped by R
// consecutive rows.  For each group we store the sorted distinct columns
// its rows touch (the union of their patterns) and an R-wide coefficient
// row of M_s per union column (zero where a row lacks the column).  The
// kernel gathers each union column once for all R rows: for the P2 node
// graph in that order a group of 4 rows has ~1.8x fewer union columns
// than nonzeros (8 rows: ~2.5x, at the price of twice the coefficients).
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstdlib>

#include "nm_internal.h"

namespace nm {
namespace {

constexpr int SORT_CAP = 8192;  // entries of one group sorted in LDS

// mode 0: count distinct columns of each group (hcount[t], -1 if the group does not fit)
// mode 1: write them (hcol + hptr[t]) and the position of every nonzero column in that list (lcol)
__global__ __launch_bounds__(256) void k_group_union(int64_t N, int rows_per_group, const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col, int mode, int32_t* hcount,
                                                   const int32_t* __restrict__ hptr, int32_t* hcol,
                                                   uint16_t* lcol) {
  __shared__ int32_t buf[SORT_CAP];
  __shared__ int32_t part[256];
  __shared__ int32_t cnt_s;
  const int64_t t = blockIdx.x;
  const int64_t r0 = t * rows_per_group;
  if (r0 >= N) return;
  const int64_t r1 = min(N, r0 + rows_per_group);
  const int32_t kb = rp[r0], ke = rp[r1];
  const int nent = ke - kb;
  if (nent > SORT_CAP) {
    if (threadIdx.x == 0 && mode == 0) hcount[t] = -1;
    return;
  }
  int n2 = 1;
  while (n2 < nent) n2 <<= 1;
  for (int i = threadIdx.x; i < n2; i += blockDim.x) buf[i] = i < nent ? col[kb + i] : INT32_MAX;
  __syncthreads();
  // bitonic sort of buf[0..n2)
  for (int k = 2; k <= n2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n2; i += blockDim.x) {
        int l = i ^ j;
        if (l > i) {
          bool up = (i & k) == 0;
          int a = buf[i], b = buf[l];
          if ((a > b) == up) {
            buf[i] = b;
            buf[l] = a;
          }
        }
      }
      __syncthreads();
    }
  // compact distinct values: each thread owns a contiguous run
  const int per = (n2 + blockDim.x - 1) / blockDim.x;
  const int i0 = threadIdx.x * per, i1 = min(n2, i0 + per);
  int c = 0;
  for (int i = i0; i < i1; ++i)
    if (buf[i] != INT32_MAX && (i == 0 || buf[i] != buf[i - 1])) ++c;
  part[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int i = 0; i < (int)blockDim.x; ++i) {
      int x = part[i];
      part[i] = s;
      s += x;
    }
    cnt_s = s;
  }
  __syncthreads();
  const int cnt = cnt_s;
  if (mode == 0) {
    if (threadIdx.x == 0) hcount[t] = cnt;
    return;
  }
  // distinct values in order, written to the group union list
  int pos = part[threadIdx.x];
  int32_t* out = hcol + hptr[t];
  for (int i = i0; i < i1; ++i)
    if (buf[i] != INT32_MAX && (i == 0 || buf[i] != buf[i - 1])) out[pos++] = buf[i];
  __syncthreads();
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) buf[i] = out[i];
  __syncthreads();
  for (int i = threadIdx.x; i < nent; i += blockDim.x) {
    const int32_t v = col[kb + i];
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (buf[mid] < v) lo = mid + 1;
      else hi = mid;
    }
    lcol[kb + i] = (uint16_t)lo;
  }
}

}  // namespace

__global__ void k_group_coef(int64_t N, int R, const int32_t* __restrict__ rp, const double* __restrict__ val,
                             const int32_t* __restrict__ gptr, const uint16_t* __restrict__ lcol,
                             double* __restrict__ coef) {
  int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= N) return;
  const int64_t g = row / R;
  const int r = (int)(row - g * R);
  for (int32_t k = rp[row]; k < rp[row + 1]; ++k) coef[((int64_t)gptr[g] + lcol[k]) * R + r] = val[k];
}

void build_row_groups(nm_pencil* P, hipStream_t st, int rows) {
  if (rows <= 0) {
    // NM_ROW_GROUPS: 0 per-row kernel only, 1 (default) grouped from 32 columns, 2 grouped at any width
    const char* env = getenv("NM_ROW_GROUPS");
    P->grouped = env ? atoi(env) : 1;
    // NM_PERSIST=1: each grouped step as one persistent launch
    const char* penv = getenv("NM_PERSIST");
    P->persist = penv ? atoi(penv) : 0;
    if (P->grouped <= 0) {
      P->grouped = 0;
      return;
    }
  }
  const char* renv = getenv("NM_GROUP_ROWS");
  const int R = rows > 0 ? rows : (renv ? atoi(renv) : 4);
  NM_REQUIRE(R == 4 || R == 8, NM_EINVAL, "row groups of 4 or 8 rows");
  const int64_t N = P->N;
  const int64_t ng = (N + R - 1) / R;
  DBuf<int32_t> cnt(ng);
  hipLaunchKernelGGL(k_group_union, dim3((unsigned)ng), dim3(256), 0, st, N, R, P->row_ptr.p, P->col.p, 0, cnt.p,
                     nullptr, nullptr, nullptr);
  std::vector<int32_t> h(ng);
  NM_HIP(hipMemcpyAsync(h.data(), cnt.p, 4 * ng, hipMemcpyDeviceToHost, st));
  NM_HIP(hipStreamSynchronize(st));
  std::vector<int32_t> ptr(ng + 1, 0);
  for (int64_t t = 0; t < ng; ++t) {
    if (h[t] < 0) {  // a group does not fit the sort: keep the per-row kernel
      P->grp_rows = 0;
      return;
    }
    ptr[t + 1] = ptr[t] + h[t];
  }
  NM_REQUIRE((int64_t)ptr[ng] * R < INT32_MAX, NM_EINVAL, "row groups too large");
  // the union list is padded by 4 entries: the grouped kernel stages it in
  // 16-byte pieces from a 4-entry boundary
  DBuf<int32_t> gptr(ng + 1), gcol((size_t)ptr[ng] + 4);
  NM_HIP(hipMemsetAsync(gcol.p + ptr[ng], 0, 4 * sizeof(int32_t), st));
  DBuf<uint16_t> lcol(std::max<int64_t>(P->nnzb, 1));
  NM_HIP(hipMemcpyAsync(gptr.p, ptr.data(), 4 * (ng + 1), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_group_union, dim3((unsigned)ng), dim3(256), 0, st, N, R, P->row_ptr.p, P->col.p, 1, nullptr,
                     gptr.p, gcol.p, lcol.p);
  DBuf<double> coef((size_t)std::max<int32_t>(ptr[ng], 1) * R);
  NM_HIP(hipMemsetAsync(coef.p, 0, coef.bytes(), st));
  hipLaunchKernelGGL(k_group_coef, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, N, R, P->row_ptr.p, P->ms.p,
                     gptr.p, lcol.p, coef.p);
  NM_HIP(hipStreamSynchronize(st));
  P->grp_rows = R;
  P->grp_ptr = std::move(gptr);
  P->grp_col = std::move(gcol);
  P->grp_coef = std::move(coef);
  if (P->ms32.p) {
    // the FP32 shadows exist already: give the new coefficients theirs
    P->grp_coef32.alloc(std::max<size_t>(P->grp_coef.n, 1));
    convert_f64_f32((int64_t)P->grp_coef.n, P->grp_coef.p, P->grp_coef32.p, st);
    NM_HIP(hipStreamSynchronize(st));
  }
}

// LDS tiles for the tiled mass-solve kernel: tiles of TR consecutive rows of
// the internal order, the sorted union of their columns (each gathered once
// per tile into LDS) and the union position of every nonzero.  TR = rows, or
// (rows 0) NM_TILE_ROWS (default 32); with rows 0 the tiles are built only
// when NM_TILES=1.
void build_tiles(nm_pencil* P, hipStream_t st, int rows) {
  P->tile_rows = 0;
  P->tile_umax = P->tile_emax = 0;
  if (rows <= 0) {
    // off by default: on the P2 planets the 4-row group kernel is faster (the
    // LDS reads of random union chunks conflict); the autotuner times both
    const char* env = getenv("NM_TILES");
    P->tiled = env ? atoi(env) : 0;
    if (P->tiled <= 0) {
      P->tiled = 0;
      return;
    }
  } else {
    P->tiled = 1;
  }
  const char* renv = getenv("NM_TILE_ROWS");
  const int TR = rows > 0 ? rows : (renv ? atoi(renv) : 32);
  NM_REQUIRE(TR >= 4 && TR <= 256, NM_EINVAL, "NM_TILE_ROWS must be in [4, 256]");
  const int64_t N = P->N;
  const int64_t nt = (N + TR - 1) / TR;
  DBuf<int32_t> cnt(nt);
  hipLaunchKernelGGL(k_group_union, dim3((unsigned)nt), dim3(256), 0, st, N, TR, P->row_ptr.p, P->col.p, 0, cnt.p,
                     nullptr, nullptr, nullptr);
  std::vector<int32_t> h(nt), rp(N + 1);
  NM_HIP(hipMemcpyAsync(h.data(), cnt.p, 4 * nt, hipMemcpyDeviceToHost, st));
  NM_HIP(hipMemcpyAsync(rp.data(), P->row_ptr.p, 4 * (N + 1), hipMemcpyDeviceToHost, st));
  NM_HIP(hipStreamSynchronize(st));
  std::vector<int32_t> ptr(nt + 1, 0);
  int umax = 0, emax = 0;
  for (int64_t t = 0; t < nt; ++t) {
    if (h[t] < 0) return;  // a tile's entries do not fit the union sort: no tiles
    ptr[t + 1] = ptr[t] + h[t];
    umax = std::max(umax, h[t]);
    emax = std::max<int>(emax, rp[std::min<int64_t>(N, (t + 1) * TR)] - rp[t * TR]);
  }
  if (umax > 65535) return;  // union positions are 16-bit
  DBuf<int32_t> tptr(nt + 1), tcol(std::max<int32_t>(ptr[nt], 1));
  DBuf<uint16_t> lcol(std::max<int64_t>(P->nnzb, 1));
  NM_HIP(hipMemcpyAsync(tptr.p, ptr.data(), 4 * (nt + 1), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_group_union, dim3((unsigned)nt), dim3(256), 0, st, N, TR, P->row_ptr.p, P->col.p, 1, nullptr,
                     tptr.p, tcol.p, lcol.p);
  NM_HIP(hipStreamSynchronize(st));
  P->tile_rows = TR;
  P->tile_umax = umax;
  P->tile_emax = emax;
  P->tile_ptr = std::move(tptr);
  P->tile_col = std::move(tcol);
  P->tile_lcol = std::move(lcol);
}

}  // namespace nm
