// Self-gravitation as an N-body problem (Sec. 5 of the paper).
//
// Bodies are the tetrahedra (at their barycentres) and the faces across
// which the density jumps: the outer surface and the fluid-solid faces (at
// their centroids).  A displacement u gives each body a charge (eqs.
// "ph1body2", "ph1surface2"):
//   tetrahedron  q_k = int_K div(rho_k u) = rho_k sum_a (int_K grad l_a) . u_a,
//   surface face q_l = int_E (nu . u) [rho]^+_- = -rho_k sum_a (int_E l_a) nu . u_a,
//   fluid-solid  q_l = int_E (nu^{f->s} . u^s) rho^s + (nu^{s->f} . u^f) rho^f,
// i.e. q = C u with C sparse (bodies x displacement DOFs).  The incremental
// potential at body i is S_i = G q_i / R_i + sum_{j != i} G q_j / |r_i - r_j|
// with the self-terms 1/R_k, 1/R_l = the mean of 1/|r - x| over the body
// (eqs. "k2local", "l2local"), and the weak form (eq. "phi1fluidsolid")
// contributes -C^T S C to the operator of eq. "eigfull".  The reference field
// of Sec. 5.1, g(x) = -G sum_k m_k (x - r_k) / |x - r_k|^3, uses the same
// bodies' masses.
//
// The N-body sums run on the device by direct tiled summation: a workgroup
// owns 256 targets and a chunk of columns; source tiles of 256 bodies
// (FP32 positions and charges) are staged in LDS; each pair's 1/r and
// products are FP32, summed over a tile in FP32 and the tile sums
// accumulated in FP64.  The ALU bounds it: per pair and column one FP32 FMA,
// plus the distance and reciprocal square root per pair.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include <cstdlib>
#include <string>

#include "nm_internal.h"

namespace {

using nm::DBuf;

__device__ __forceinline__ int64_t gtid() { return nm_xcd_block() * blockDim.x + threadIdx.x; }

// Y[r][c] = s * sum_k val[k] X[col[k]][c], lanes (row, column)
__global__ void k_csr_cols(int64_t rows, int nc, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           const double* __restrict__ val, const double* __restrict__ X, double s,
                           double* __restrict__ Y, float* __restrict__ Y32) {
  const int64_t g = gtid();
  if (g >= rows * nc) return;
  const int64_t r = g / nc;
  const int c = (int)(g - r * nc);
  double acc = 0.0;
  for (int32_t k = rp[r]; k < rp[r + 1]; ++k) acc += val[k] * X[(int64_t)ci[k] * nc + c];
  acc *= s;
  if (Y) Y[g] = acc;
  if (Y32) Y32[g] = (float)acc;
}

// Y[r][c] += sum_k val[k] X[col[k]][c]
__global__ void k_csr_cols_add(int64_t rows, int nc, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                               const double* __restrict__ val, const double* __restrict__ X, double* __restrict__ Y) {
  const int64_t g = gtid();
  if (g >= rows * nc) return;
  const int64_t r = g / nc;
  const int c = (int)(g - r * nc);
  double acc = 0.0;
  for (int32_t k = rp[r]; k < rp[r + 1]; ++k) acc += val[k] * X[(int64_t)ci[k] * nc + c];
  Y[g] += acc;
}

constexpr int NB_TILE = 256;

// phi[i][c] = G (q[i][c] invR[i] + sum_{j != i} q[j][c] / |r_i - r_j|), columns
// c0 .. c0 + CB of nc; FP32 pair terms, FP64 sum of the per-tile FP32 sums
template <int CB>
__global__ __launch_bounds__(256) void k_nbody(int64_t nb, int nc, const float4* __restrict__ pos,
                                               const float* __restrict__ q, const double* __restrict__ invR,
                                               const double* __restrict__ q64, double G, double* __restrict__ phi) {
  __shared__ float4 s_pos[NB_TILE];
  __shared__ float s_q[NB_TILE][CB];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int c0 = blockIdx.y * CB;
  const bool has = i < nb;
  const float4 pi = has ? pos[i] : make_float4(0.f, 0.f, 0.f, 0.f);
  double acc[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) acc[c] = 0.0;
  for (int64_t j0 = 0; j0 < nb; j0 += NB_TILE) {
    __syncthreads();
    {
      const int64_t j = j0 + threadIdx.x;
      s_pos[threadIdx.x] = j < nb ? pos[j] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int c = 0; c < CB; ++c) s_q[threadIdx.x][c] = (j < nb && c0 + c < nc) ? q[j * nc + c0 + c] : 0.f;
    }
    __syncthreads();
    float t[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) t[c] = 0.f;
    const int lim = (int)min<int64_t>(NB_TILE, nb - j0);
    for (int jj = 0; jj < lim; ++jj) {
      const float4 pj = s_pos[jj];
      const float dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
      const float r2 = dx * dx + dy * dy + dz * dz;
      // the self pair (r2 == 0 only for j == i: bodies are distinct points) adds nothing here
      const float ir = (j0 + jj == i) ? 0.f : rsqrtf(r2);
#pragma unroll
      for (int c = 0; c < CB; ++c) t[c] += s_q[jj][c] * ir;
    }
#pragma unroll
    for (int c = 0; c < CB; ++c) acc[c] += (double)t[c];
  }
  if (!has) return;
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    if (c0 + c >= nc) break;
    phi[i * nc + c0 + c] = G * (acc[c] + invR[i] * q64[i * nc + c0 + c]);
  }
}

// The same sums register-blocked: each lane owns TPL targets (i0 + t 256 +
// lane, so the loads stay coalesced) and reuses every staged source (its
// position and CB charges, read from LDS as float4s) for all of them; the
// inner loop over a full tile is unrolled, and only tiles that hold one of
// the workgroup's own targets test for the self pair.  The sources are split
// into runs (blockIdx.z) so that a launch has enough workgroups to fill the
// chip even for few columns; each run writes its FP64 partial sums, which
// k_nbody_reduce adds in run order.  CB is a multiple of 4.
template <int CB, int TPL>
__global__ __launch_bounds__(256) void k_nbody_rb(int64_t nb, int nc, const float4* __restrict__ pos,
                                                  const float* __restrict__ q, int64_t span,
                                                  double* __restrict__ part) {
  constexpr int CQ = CB / 4;
  __shared__ float4 s_pos[NB_TILE];
  __shared__ float4 s_q[NB_TILE][CQ];
  const int64_t i0 = (int64_t)blockIdx.x * (256 * TPL);
  const int c0 = blockIdx.y * CB;
  int64_t ii[TPL];
  float4 pi[TPL];
#pragma unroll
  for (int t = 0; t < TPL; ++t) {
    ii[t] = i0 + t * 256 + threadIdx.x;
    pi[t] = ii[t] < nb ? pos[ii[t]] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  double acc[TPL][CB];
#pragma unroll
  for (int t = 0; t < TPL; ++t)
#pragma unroll
    for (int c = 0; c < CB; ++c) acc[t][c] = 0.0;
  // this workgroup's run of sources: [js, je), span a multiple of NB_TILE
  const int64_t js = (int64_t)blockIdx.z * span, je = min<int64_t>(nb, js + span);
  for (int64_t j0 = js; j0 < je; j0 += NB_TILE) {
    __syncthreads();
    {
      const int64_t j = j0 + threadIdx.x;
      s_pos[threadIdx.x] = j < nb ? pos[j] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int cq = 0; cq < CQ; ++cq) {
        float v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c = c0 + 4 * cq + u;
          v[u] = (j < nb && c < nc) ? q[j * nc + c] : 0.f;
        }
        s_q[threadIdx.x][cq] = make_float4(v[0], v[1], v[2], v[3]);
      }
    }
    __syncthreads();
    float tsum[TPL][CB];
#pragma unroll
    for (int t = 0; t < TPL; ++t)
#pragma unroll
      for (int c = 0; c < CB; ++c) tsum[t][c] = 0.f;
    const int lim = (int)min<int64_t>(NB_TILE, nb - j0);
    const bool own = j0 < i0 + 256 * TPL && j0 + NB_TILE > i0;
    if (!own && lim == NB_TILE) {
#pragma unroll 4
      for (int jj = 0; jj < NB_TILE; ++jj) {
        const float4 pj = s_pos[jj];
        float qq[CB];
#pragma unroll
        for (int cq = 0; cq < CQ; ++cq) {
          const float4 v = s_q[jj][cq];
          qq[4 * cq] = v.x; qq[4 * cq + 1] = v.y; qq[4 * cq + 2] = v.z; qq[4 * cq + 3] = v.w;
        }
#pragma unroll
        for (int t = 0; t < TPL; ++t) {
          const float dx = pi[t].x - pj.x, dy = pi[t].y - pj.y, dz = pi[t].z - pj.z;
          const float ir = rsqrtf(dx * dx + dy * dy + dz * dz);
#pragma unroll
          for (int c = 0; c < CB; ++c) tsum[t][c] += qq[c] * ir;
        }
      }
    } else {
      for (int jj = 0; jj < lim; ++jj) {
        const float4 pj = s_pos[jj];
        float qq[CB];
#pragma unroll
        for (int cq = 0; cq < CQ; ++cq) {
          const float4 v = s_q[jj][cq];
          qq[4 * cq] = v.x; qq[4 * cq + 1] = v.y; qq[4 * cq + 2] = v.z; qq[4 * cq + 3] = v.w;
        }
#pragma unroll
        for (int t = 0; t < TPL; ++t) {
          const float dx = pi[t].x - pj.x, dy = pi[t].y - pj.y, dz = pi[t].z - pj.z;
          const float ir = (j0 + jj == ii[t]) ? 0.f : rsqrtf(dx * dx + dy * dy + dz * dz);
#pragma unroll
          for (int c = 0; c < CB; ++c) tsum[t][c] += qq[c] * ir;
        }
      }
    }
#pragma unroll
    for (int t = 0; t < TPL; ++t)
#pragma unroll
      for (int c = 0; c < CB; ++c) acc[t][c] += (double)tsum[t][c];
  }
  // partial sums of this source run: part[z][i][c]
  double* pz = part + (int64_t)blockIdx.z * nb * nc;
#pragma unroll
  for (int t = 0; t < TPL; ++t) {
    if (ii[t] >= nb) continue;
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      if (c0 + c >= nc) break;
      pz[ii[t] * nc + c0 + c] = acc[t][c];
    }
  }
}

// phi = G (sum over the source runs in order + invR q): deterministic
__global__ void k_nbody_reduce(int64_t nb, int nc, int nsplit, const double* __restrict__ part,
                               const double* __restrict__ invR, const double* __restrict__ q64, double G,
                               double* __restrict__ phi) {
  const int64_t g = gtid();
  if (g >= nb * nc) return;
  double s = 0.0;
  for (int z = 0; z < nsplit; ++z) s += part[(int64_t)z * nb * nc + g];
  phi[g] = G * (s + invR[g / nc] * q64[g]);
}

// reference field g(x_p) = -G sum_k m_k (x_p - r_k) / |x_p - r_k|^3 (FP32 pairs, FP64 tile sums)
__global__ __launch_bounds__(256) void k_nbody_field(int64_t np, const double* __restrict__ pts, int64_t nm,
                                                     const float4* __restrict__ pos, const float* __restrict__ mass,
                                                     double G, double* __restrict__ g) {
  __shared__ float4 s_pos[NB_TILE];
  __shared__ float s_m[NB_TILE];
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool has = p < np;
  const float px = has ? (float)pts[3 * p] : 0.f, py = has ? (float)pts[3 * p + 1] : 0.f,
              pz = has ? (float)pts[3 * p + 2] : 0.f;
  double ax = 0.0, ay = 0.0, az = 0.0;
  for (int64_t j0 = 0; j0 < nm; j0 += NB_TILE) {
    __syncthreads();
    const int64_t j = j0 + threadIdx.x;
    s_pos[threadIdx.x] = j < nm ? pos[j] : make_float4(0.f, 0.f, 0.f, 0.f);
    s_m[threadIdx.x] = j < nm ? mass[j] : 0.f;
    __syncthreads();
    float tx = 0.f, ty = 0.f, tz = 0.f;
    const int lim = (int)min<int64_t>(NB_TILE, nm - j0);
    for (int jj = 0; jj < lim; ++jj) {
      const float4 pj = s_pos[jj];
      const float dx = px - pj.x, dy = py - pj.y, dz = pz - pj.z;
      const float r2 = dx * dx + dy * dy + dz * dz;
      const float ir = r2 > 0.f ? rsqrtf(r2) : 0.f;
      const float w = s_m[jj] * ir * ir * ir;
      tx += w * dx;
      ty += w * dy;
      tz += w * dz;
    }
    ax += tx;
    ay += ty;
    az += tz;
  }
  if (!has) return;
  g[3 * p] = -G * ax;
  g[3 * p + 1] = -G * ay;
  g[3 * p + 2] = -G * az;
}

// mean of 1/|x - r_k| over tetrahedron k from its barycentre r_k: the four
// cones from r_k over the faces, int_cone 1/|x - r| = (h/2) int_F dA/|y - r|,
// each face integral by the collapsed Gauss rule (s, t, w) of nq points
__global__ void k_tet_selfterm(int64_t T, const double* __restrict__ xyz, const int32_t* __restrict__ tet, int nq,
                               const double* __restrict__ qs, const double* __restrict__ qt,
                               const double* __restrict__ qw, double* __restrict__ out) {
  const int64_t k = gtid();
  if (k >= T) return;
  double X[4][3], r[3] = {0, 0, 0};
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 3; ++c) {
      X[a][c] = xyz[3 * (int64_t)tet[4 * k + a] + c];
      r[c] += 0.25 * X[a][c];
    }
  double e1[3], e2[3], e3[3];
  for (int c = 0; c < 3; ++c) {
    e1[c] = X[1][c] - X[0][c];
    e2[c] = X[2][c] - X[0][c];
    e3[c] = X[3][c] - X[0][c];
  }
  const double vol = fabs(e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) - e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
                          e1[2] * (e2[0] * e3[1] - e2[1] * e3[0])) / 6.0;
  double tot = 0.0;
  for (int f = 0; f < 4; ++f) {
    const int a = f == 0 ? 1 : 0, b = f <= 1 ? 2 : 1, c = f <= 2 ? 3 : 2;  // the face opposite vertex f
    double u[3], v[3], n[3];
    for (int q = 0; q < 3; ++q) {
      u[q] = X[b][q] - X[a][q];
      v[q] = X[c][q] - X[a][q];
    }
    n[0] = u[1] * v[2] - u[2] * v[1];
    n[1] = u[2] * v[0] - u[0] * v[2];
    n[2] = u[0] * v[1] - u[1] * v[0];
    const double a2 = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    const double h = fabs((r[0] - X[a][0]) * n[0] + (r[1] - X[a][1]) * n[1] + (r[2] - X[a][2]) * n[2]) / a2;
    double s = 0.0;
    for (int p = 0; p < nq; ++p) {
      double y[3];
      for (int q = 0; q < 3; ++q) y[q] = X[a][q] + qs[p] * u[q] + qt[p] * v[q] - r[q];
      s += qw[p] / sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    }
    tot += 0.5 * h * a2 * s;
  }
  out[k] = tot / vol;
}

// mean of 1/|x - P| over the triangle ABC, P (the centroid) in its plane:
// three pieces with apex P; over a piece with far edge XY the radial
// integral is the distance d to the edge's line: d (asinh(s2) - asinh(s1))
double tri_selfterm(const double* A, const double* B, const double* C) {
  double P[3];
  for (int q = 0; q < 3; ++q) P[q] = (A[q] + B[q] + C[q]) / 3.0;
  auto piece = [&](const double* X, const double* Y) {
    double e[3], L = 0;
    for (int q = 0; q < 3; ++q) {
      e[q] = Y[q] - X[q];
      L += e[q] * e[q];
    }
    L = std::sqrt(L);
    for (int q = 0; q < 3; ++q) e[q] /= L;
    double px = 0;
    for (int q = 0; q < 3; ++q) px += (P[q] - X[q]) * e[q];
    double foot[3], d = 0;
    for (int q = 0; q < 3; ++q) {
      foot[q] = X[q] + px * e[q];
      d += (P[q] - foot[q]) * (P[q] - foot[q]);
    }
    d = std::sqrt(d);
    if (d <= 0) return 0.0;
    double s1 = 0, s2 = 0;
    for (int q = 0; q < 3; ++q) {
      s1 += (X[q] - foot[q]) * e[q];
      s2 += (Y[q] - foot[q]) * e[q];
    }
    return d * (std::asinh(s2 / d) - std::asinh(s1 / d));
  };
  double u[3], v[3];
  for (int q = 0; q < 3; ++q) {
    u[q] = B[q] - A[q];
    v[q] = C[q] - A[q];
  }
  const double n0 = u[1] * v[2] - u[2] * v[1], n1 = u[2] * v[0] - u[0] * v[2], n2 = u[0] * v[1] - u[1] * v[0];
  const double area = 0.5 * std::sqrt(n0 * n0 + n1 * n1 + n2 * n2);
  return std::fabs(piece(A, B) + piece(B, C) + piece(C, A)) / area;
}

struct Trip {
  int64_t r, c;
  double v;
};

void csr_from(std::vector<Trip>& t, int64_t rows, std::vector<int32_t>& ptr, std::vector<int32_t>& col,
              std::vector<double>& val) {
  std::sort(t.begin(), t.end(), [](const Trip& a, const Trip& b) { return a.r != b.r ? a.r < b.r : a.c < b.c; });
  ptr.assign(rows + 1, 0);
  col.clear();
  val.clear();
  for (size_t i = 0; i < t.size();) {
    size_t j = i;
    double s = 0;
    while (j < t.size() && t[j].r == t[i].r && t[j].c == t[i].c) s += t[j++].v;
    col.push_back((int32_t)t[i].c);
    val.push_back(s);
    ptr[t[i].r + 1]++;
    i = j;
  }
  for (int64_t r = 0; r < rows; ++r) ptr[r + 1] += ptr[r];
}

}  // namespace

struct nm_selfgrav {
  const nm_pencil* P = nullptr;
  int64_t nbody = 0, ntet = 0, nface = 0;
  double G = 0;
  DBuf<float4> pos;        // body positions (FP32), tetrahedra first
  DBuf<float> mass32;      // element masses (FP32) for the reference field
  DBuf<double> invR;       // 1/R_i
  DBuf<int32_t> c_ptr, c_col, ct_ptr, ct_col;  // C (bodies x internal DOF) and C^T
  DBuf<double> c_val, ct_val;
  // work buffers of apply (sized for the widest block seen; one caller at a time)
  int wcols = 0;
  DBuf<double> q64, phi, part;
  DBuf<float> q32;
  void ensure_part(size_t elems) {
    if (part.n < elems) part.alloc(elems);
  }
  void ensure(int nc) {
    if (nc <= wcols) return;
    q64.alloc((size_t)nbody * nc);
    phi.alloc((size_t)nbody * nc);
    q32.alloc((size_t)nbody * nc);
    wcols = nc;
  }
};

namespace nm {

// F -= C^T S C X (internal node order, FP64, [N][3 nc])
void selfgrav_add(const nm_selfgrav* sgc, int nc, const double* X, double* F, hipStream_t st) {
  nm_selfgrav* sg = const_cast<nm_selfgrav*>(sgc);
  sg->ensure(nc);
  const int64_t nb = sg->nbody, n = 3 * sg->P->N;
  hipLaunchKernelGGL(k_csr_cols, dim3(grid_for(nb * nc)), dim3(256), 0, st, nb, nc, sg->c_ptr.p, sg->c_col.p,
                     sg->c_val.p, X, 1.0, sg->q64.p, sg->q32.p);
  // kernel: NM_NBODY=simple (one target per lane, for comparison) or the
  // default: two targets per lane, LDS-staged sources split into runs
  const char* kn = std::getenv("NM_NBODY");
  constexpr int CB = 8, TPL = 2;
  if (kn && std::string(kn) == "simple") {
    dim3 grid((unsigned)((nb + 255) / 256), (unsigned)((nc + CB - 1) / CB));
    hipLaunchKernelGGL((k_nbody<CB>), grid, dim3(256), 0, st, nb, nc, sg->pos.p, sg->q32.p, sg->invR.p, sg->q64.p,
                       sg->G, sg->phi.p);
  } else {
    const int64_t bx = (nb + 256 * TPL - 1) / (256 * TPL), by = (nc + CB - 1) / CB;
    const int64_t tiles = (nb + NB_TILE - 1) / NB_TILE;
    // about 2048 workgroups, at least one source tile per run, at most 16 runs
    const int64_t want = std::min<int64_t>(16, std::max<int64_t>(1, (2048 + bx * by - 1) / (bx * by)));
    const int64_t span = NB_TILE * ((tiles + want - 1) / want);
    const int nsplit = (int)((nb + span - 1) / span);
    sg->ensure_part((size_t)nsplit * nb * nc);
    dim3 grid((unsigned)bx, (unsigned)by, (unsigned)nsplit);
    hipLaunchKernelGGL((k_nbody_rb<CB, TPL>), grid, dim3(256), 0, st, nb, nc, sg->pos.p, sg->q32.p, span,
                       sg->part.p);
    hipLaunchKernelGGL(k_nbody_reduce, dim3(grid_for(nb * nc)), dim3(256), 0, st, nb, nc, nsplit, sg->part.p,
                       sg->invR.p, sg->q64.p, sg->G, sg->phi.p);
  }
  // F -= C^T phi: the scattered term is added with the sign folded into phi's use
  hipLaunchKernelGGL(k_csr_cols_add, dim3(grid_for(n * nc)), dim3(256), 0, st, n, nc, sg->ct_ptr.p, sg->ct_col.p,
                     sg->ct_val.p, sg->phi.p, F);
}

}  // namespace nm

extern "C" {

nm_status nm_selfgrav_build(nm_pencil* p, const nm_mesh* mesh, const nm_material* mat, double G, void* stream,
                            nm_selfgrav** out) {
  NM_TRY({
    NM_REQUIRE(p && mesh && mat && out && G > 0, NM_EINVAL, "invalid arguments");
    NM_REQUIRE(mesh->n_vert == p->V && mesh->n_tet == p->T && mesh->disp_order == p->disp_order, NM_EINVAL,
               "the mesh is not the pencil's");
    *out = nullptr;
    hipStream_t st = (hipStream_t)stream;
    const int64_t V = mesh->n_vert, T = mesh->n_tet, N = p->N, n = 3 * N;
    const int order = mesh->disp_order, nd = order == 2 ? 10 : 4;
    const double* xyz = mesh->xyz;
    const int32_t* tet = mesh->tet;
    // canonical displacement node of each (geometric node, side), then its internal index
    std::vector<int32_t> ng(N), perm(N);
    NM_HIP(hipMemcpyAsync(ng.data(), p->node_geom.p, 4 * N, hipMemcpyDeviceToHost, st));
    NM_HIP(hipMemcpyAsync(perm.data(), p->perm.p, 4 * N, hipMemcpyDeviceToHost, st));
    NM_HIP(hipStreamSynchronize(st));
    std::vector<int32_t> sol(p->n_geom, -1), flu(p->n_geom, -1);
    for (int64_t i = 0; i < N; ++i) (i < p->n_solid ? sol : flu)[ng[i]] = perm[i];
    // geometric nodes of each element: vertices, then edges by the sorted (min, max) rule
    static const int E6[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    std::vector<uint64_t> ekeys;
    if (order == 2) {
      ekeys.reserve(6 * T);
      for (int64_t t = 0; t < T; ++t)
        for (int e = 0; e < 6; ++e) {
          uint64_t a = (uint32_t)tet[4 * t + E6[e][0]], b = (uint32_t)tet[4 * t + E6[e][1]];
          ekeys.push_back(std::min(a, b) << 32 | std::max(a, b));
        }
      std::sort(ekeys.begin(), ekeys.end());
      ekeys.erase(std::unique(ekeys.begin(), ekeys.end()), ekeys.end());
    }
    auto geom_of = [&](int64_t t, int a) -> int64_t {
      if (a < 4) return tet[4 * t + a];
      uint64_t x = (uint32_t)tet[4 * t + E6[a - 4][0]], y = (uint32_t)tet[4 * t + E6[a - 4][1]];
      const uint64_t k = std::min(x, y) << 32 | std::max(x, y);
      return V + (int64_t)(std::lower_bound(ekeys.begin(), ekeys.end(), k) - ekeys.begin());
    };
    auto dnode = [&](int64_t t, int a) -> int64_t {
      const int64_t g = geom_of(t, a);
      const int32_t d = mesh->region[t] == 0 ? sol[g] : flu[g];
      NM_REQUIRE(d >= 0, NM_EBADMESH, "element node without a displacement copy");
      return d;
    };
    std::vector<Trip> tc;
    tc.reserve((size_t)T * nd * 3 + 64);
    std::vector<double> bpos;  // body positions
    bpos.reserve(3 * T);
    std::vector<float> masses(T);
    // tetrahedra: q_k = rho_k sum_a (int_K grad l_a) . u_a; int_K grad l_a = |K| grad lambda_a (P1),
    // 0 at P2 vertices and |K| (grad lambda_i + grad lambda_j) at the P2 node of edge (i, j)
    for (int64_t t = 0; t < T; ++t) {
      double X[4][3];
      for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 3; ++c) X[a][c] = xyz[3 * (int64_t)tet[4 * t + a] + c];
      double J[3][3];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) J[r][c] = X[c + 1][r] - X[0][r];  // columns: edges from vertex 0
      const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                         J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
      NM_REQUIRE(det > 0, NM_EBADMESH, "tetrahedron " + std::to_string(t) + " has J <= 0");
      double inv[3][3];  // rows: grad lambda_1..3
      inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
      inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
      inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
      inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
      inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
      inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
      inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
      inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
      inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
      double gl[4][3];
      for (int c = 0; c < 3; ++c) {
        gl[1][c] = inv[0][c];
        gl[2][c] = inv[1][c];
        gl[3][c] = inv[2][c];
        gl[0][c] = -(gl[1][c] + gl[2][c] + gl[3][c]);
      }
      const double vol = det / 6.0, rho = mat->rho[t];
      masses[t] = (float)(rho * vol);
      for (int a = 0; a < nd; ++a) {
        double gi[3] = {0, 0, 0};
        if (order == 1) {
          for (int c = 0; c < 3; ++c) gi[c] = vol * gl[a][c];
        } else if (a >= 4) {
          for (int c = 0; c < 3; ++c) gi[c] = vol * (gl[E6[a - 4][0]][c] + gl[E6[a - 4][1]][c]);
        } else {
          continue;
        }
        const int64_t d = dnode(t, a);
        for (int c = 0; c < 3; ++c) tc.push_back({t, 3 * d + c, rho * gi[c]});
      }
      for (int c = 0; c < 3; ++c) bpos.push_back(0.25 * (X[0][c] + X[1][c] + X[2][c] + X[3][c]));
    }
    // faces: keys of the four faces of every tetrahedron (face f opposite vertex f)
    static const int FV[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    struct FK {
      int32_t v[3];
      int64_t t;
      int f;
    };
    std::vector<FK> fk(4 * T);
    for (int64_t t = 0; t < T; ++t)
      for (int f = 0; f < 4; ++f) {
        FK k;
        for (int q = 0; q < 3; ++q) k.v[q] = tet[4 * t + FV[f][q]];
        std::sort(k.v, k.v + 3);
        k.t = t;
        k.f = f;
        fk[4 * t + f] = k;
      }
    std::sort(fk.begin(), fk.end(), [](const FK& a, const FK& b) {
      for (int q = 0; q < 3; ++q)
        if (a.v[q] != b.v[q]) return a.v[q] < b.v[q];
      return a.t < b.t;
    });
    std::vector<double> tri_invR;
    int64_t row = T;
    // face-local nodes of face f of a tetrahedron: its three vertices, then (P2) its edges
    auto face_nodes = [&](int f, int* loc) {
      const int a = FV[f][0], b = FV[f][1], c = FV[f][2];
      loc[0] = a;
      loc[1] = b;
      loc[2] = c;
      if (order == 2) {
        auto eid = [&](int x, int y) {
          for (int e = 0; e < 6; ++e)
            if ((E6[e][0] == x && E6[e][1] == y) || (E6[e][0] == y && E6[e][1] == x)) return 4 + e;
          return -1;
        };
        loc[3] = eid(a, b);
        loc[4] = eid(a, c);
        loc[5] = eid(b, c);
      }
    };
    const int nfn = order == 2 ? 6 : 3;
    // int_E l_a / |E|: 1/3 at P1 nodes; 0 at P2 vertices and 1/3 at P2 edge nodes
    auto fint = [&](int q) { return order == 1 ? 1.0 / 3.0 : (q < 3 ? 0.0 : 1.0 / 3.0); };
    auto face_geo = [&](int64_t t, int f, double* nu, double& area, double* cen, double (*Xf)[3]) {
      double X[4][3];
      for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 3; ++c) X[a][c] = xyz[3 * (int64_t)tet[4 * t + a] + c];
      const int a = FV[f][0], b = FV[f][1], c = FV[f][2];
      double u[3], v[3];
      for (int q = 0; q < 3; ++q) {
        u[q] = X[b][q] - X[a][q];
        v[q] = X[c][q] - X[a][q];
        cen[q] = (X[a][q] + X[b][q] + X[c][q]) / 3.0;
        Xf[0][q] = X[a][q];
        Xf[1][q] = X[b][q];
        Xf[2][q] = X[c][q];
      }
      nu[0] = u[1] * v[2] - u[2] * v[1];
      nu[1] = u[2] * v[0] - u[0] * v[2];
      nu[2] = u[0] * v[1] - u[1] * v[0];
      const double l = std::sqrt(nu[0] * nu[0] + nu[1] * nu[1] + nu[2] * nu[2]);
      area = 0.5 * l;
      double out_dir = 0;
      for (int q = 0; q < 3; ++q) {
        nu[q] /= l;
        out_dir += nu[q] * (X[a][q] - X[f][q]);  // vertex f lies opposite the face
      }
      if (out_dir < 0)
        for (int q = 0; q < 3; ++q) nu[q] = -nu[q];
    };
    for (size_t i = 0; i < fk.size();) {
      size_t j = i + 1;
      while (j < fk.size() && fk[j].v[0] == fk[i].v[0] && fk[j].v[1] == fk[i].v[1] && fk[j].v[2] == fk[i].v[2]) ++j;
      const int cnt = (int)(j - i);
      double nu[3], area, cen[3], Xf[3][3];
      int loc[6];
      if (cnt == 1) {
        // outer surface: [rho]^+_- = -rho_t, nu outward
        const int64_t t = fk[i].t;
        face_geo(t, fk[i].f, nu, area, cen, Xf);
        face_nodes(fk[i].f, loc);
        for (int q = 0; q < nfn; ++q) {
          const double w = fint(q);
          if (w == 0) continue;
          const int64_t d = dnode(t, loc[q]);
          for (int c = 0; c < 3; ++c) tc.push_back({row, 3 * d + c, -mat->rho[t] * area * w * nu[c]});
        }
      } else if (cnt == 2 && mesh->region[fk[i].t] != mesh->region[fk[i + 1].t]) {
        // fluid-solid: (nu^{f->s} . u^s) rho^s + (nu^{s->f} . u^f) rho^f
        const int64_t ts = mesh->region[fk[i].t] == 0 ? fk[i].t : fk[i + 1].t;
        const int fs_ = mesh->region[fk[i].t] == 0 ? fk[i].f : fk[i + 1].f;
        const int64_t tf = ts == fk[i].t ? fk[i + 1].t : fk[i].t;
        face_geo(ts, fs_, nu, area, cen, Xf);  // nu: outward from the solid, s -> f
        face_nodes(fs_, loc);
        for (int q = 0; q < nfn; ++q) {
          const double w = fint(q);
          if (w == 0) continue;
          const int64_t g = geom_of(ts, loc[q]);
          const int64_t ds = sol[g], df = flu[g];
          NM_REQUIRE(ds >= 0 && df >= 0, NM_EBADMESH, "fluid-solid node without both copies");
          for (int c = 0; c < 3; ++c) {
            tc.push_back({row, 3 * ds + c, -mat->rho[ts] * area * w * nu[c]});  // nu^{f->s} = -nu
            tc.push_back({row, 3 * df + c, mat->rho[tf] * area * w * nu[c]});   // nu^{s->f} = nu
          }
        }
      } else {
        i = j;
        continue;
      }
      for (int c = 0; c < 3; ++c) bpos.push_back(cen[c]);
      tri_invR.push_back(tri_selfterm(Xf[0], Xf[1], Xf[2]));
      ++row;
      i = j;
    }
    nm_selfgrav* sg = new nm_selfgrav();
    try {
      sg->P = p;
      sg->G = G;
      sg->ntet = T;
      sg->nbody = row;
      sg->nface = row - T;
      std::vector<int32_t> cp, cc, tp, tcn;
      std::vector<double> cv, tv;
      csr_from(tc, row, cp, cc, cv);
      std::vector<Trip> tt(tc.size());
      for (size_t k = 0; k < tc.size(); ++k) tt[k] = {tc[k].c, tc[k].r, tc[k].v};
      csr_from(tt, n, tp, tcn, tv);
      auto up = [&](auto& buf, const auto& h) {
        buf.alloc(std::max<size_t>(h.size(), 1));
        if (!h.empty()) NM_HIP(hipMemcpyAsync(buf.p, h.data(), sizeof(h[0]) * h.size(), hipMemcpyHostToDevice, st));
      };
      up(sg->c_ptr, cp);
      up(sg->c_col, cc);
      up(sg->c_val, cv);
      up(sg->ct_ptr, tp);
      up(sg->ct_col, tcn);
      // C^T enters as -C^T S C: store -C^T so the scatter adds
      for (auto& x : tv) x = -x;
      up(sg->ct_val, tv);
      std::vector<float4> p4(row);
      for (int64_t b = 0; b < row; ++b)
        p4[b] = make_float4((float)bpos[3 * b], (float)bpos[3 * b + 1], (float)bpos[3 * b + 2], 0.f);
      up(sg->pos, p4);
      up(sg->mass32, masses);
      // self-terms: tetrahedra on the device (collapsed 24 x 24 Gauss rule), faces closed form
      const int ng1 = 24;
      std::vector<double> gx(ng1), gw(ng1);
      for (int i = 0; i < ng1; ++i) {  // Gauss-Legendre nodes on [0, 1] by Newton iteration on P_n
        double x = std::cos(M_PI * (i + 0.75) / (ng1 + 0.5)), dp = 0;
        for (int it = 0; it < 100; ++it) {
          double p0 = 1, p1 = x;
          for (int k = 2; k <= ng1; ++k) {
            const double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = p2;
          }
          dp = ng1 * (x * p1 - p0) / (x * x - 1);
          const double dx = p1 / dp;
          x -= dx;
          if (std::fabs(dx) < 1e-16) break;
        }
        gx[i] = 0.5 * (x + 1);
        gw[i] = 1.0 / ((1 - x * x) * dp * dp);  // = 0.5 * 2 / ((1 - x^2) P'^2)
      }
      std::vector<double> qs, qt, qw;
      for (int i = 0; i < ng1; ++i)
        for (int j = 0; j < ng1; ++j) {
          qs.push_back(gx[i]);
          qt.push_back(gx[j] * (1 - gx[i]));
          qw.push_back(gw[i] * gw[j] * (1 - gx[i]));
        }
      DBuf<double> dxyz(3 * V), dqs(qs.size()), dqt(qt.size()), dqw(qw.size());
      DBuf<int32_t> dtet(4 * T);
      NM_HIP(hipMemcpyAsync(dxyz.p, xyz, 8 * 3 * V, hipMemcpyHostToDevice, st));
      NM_HIP(hipMemcpyAsync(dtet.p, tet, 4 * 4 * T, hipMemcpyHostToDevice, st));
      NM_HIP(hipMemcpyAsync(dqs.p, qs.data(), 8 * qs.size(), hipMemcpyHostToDevice, st));
      NM_HIP(hipMemcpyAsync(dqt.p, qt.data(), 8 * qt.size(), hipMemcpyHostToDevice, st));
      NM_HIP(hipMemcpyAsync(dqw.p, qw.data(), 8 * qw.size(), hipMemcpyHostToDevice, st));
      sg->invR.alloc(row);
      hipLaunchKernelGGL(k_tet_selfterm, dim3(nm::grid_for(T)), dim3(256), 0, st, T, dxyz.p, dtet.p, (int)qs.size(),
                         dqs.p, dqt.p, dqw.p, sg->invR.p);
      if (row > T)
        NM_HIP(hipMemcpyAsync(sg->invR.p + T, tri_invR.data(), 8 * (row - T), hipMemcpyHostToDevice, st));
      NM_HIP(hipStreamSynchronize(st));
      NM_HIP(hipGetLastError());
    } catch (...) {
      delete sg;
      throw;
    }
    *out = sg;
  })
}

nm_status nm_selfgrav_info(const nm_selfgrav* sg, int64_t* nbody, int64_t* ntet, int64_t* nface, double* inv_R) {
  NM_TRY({
    NM_REQUIRE(sg, NM_EINVAL, "null argument");
    if (nbody) *nbody = sg->nbody;
    if (ntet) *ntet = sg->ntet;
    if (nface) *nface = sg->nface;
    if (inv_R) NM_HIP(hipMemcpy(inv_R, sg->invR.p, 8 * sg->nbody, hipMemcpyDeviceToHost));
  })
}

nm_status nm_selfgrav_apply(const nm_selfgrav* sg, int32_t ncols, const double* X, double* Y, void* stream) {
  NM_TRY({
    NM_REQUIRE(sg && X && Y && X != Y, NM_EINVAL, "invalid arguments");
    const nm_pencil* P = sg->P;
    nm::check_block(3 * P->N, ncols);
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = 3 * P->N;
    DBuf<double> xi((size_t)n * ncols), yi((size_t)n * ncols);
    nm::permute_rows(P->N, 3 * ncols, X, xi.p, P->iperm.p, 8, st);
    NM_HIP(hipMemsetAsync(yi.p, 0, yi.bytes(), st));
    nm::selfgrav_add(sg, ncols, xi.p, yi.p, st);
    nm::permute_rows(P->N, 3 * ncols, yi.p, Y, P->perm.p, 8, st);
    NM_HIP(hipStreamSynchronize(st));
    NM_HIP(hipGetLastError());
  })
}

nm_status nm_selfgrav_field(const nm_selfgrav* sg, int64_t npts, const double* pts, double* g, void* stream) {
  NM_TRY({
    NM_REQUIRE(sg && pts && g && npts > 0, NM_EINVAL, "invalid arguments");
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_nbody_field, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, npts, pts, sg->ntet,
                       sg->pos.p, sg->mass32.p, sg->G, g);
    NM_HIP(hipStreamSynchronize(st));
    NM_HIP(hipGetLastError());
  })
}

nm_status nm_pencil_attach_selfgrav(nm_pencil* p, const nm_selfgrav* sg) {
  NM_TRY({
    NM_REQUIRE(p && (!sg || sg->P == p), NM_EINVAL, "the self-gravitation belongs to another pencil");
    p->selfgrav = sg;
  })
}

void nm_selfgrav_free(nm_selfgrav* sg) { delete sg; }

}  // extern "C"
