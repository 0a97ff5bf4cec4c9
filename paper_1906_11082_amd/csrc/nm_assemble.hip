// Numbering, CSR patterns and matrix values of the pencil, on the device.
//
// Paper: table of implicit matrix definitions (Sec. 4.2), element formulas
// of Appendix A, non-conforming fluid-solid coupling (Sec. 4.1).  The
// paper assembles "using standard techniques"; here every pattern is the
// set of unique (row, col) keys of all element contributions, found by a
// stable radix sort of 64-bit keys, and every value is the sum of its
// contributions in sorted (= element) order: no floating-point atomics, so
// the matrices are bitwise reproducible.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>

#include "nm_internal.h"

namespace nm {
namespace {

__constant__ int c_edge[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
__constant__ int c_facev[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
__constant__ int c_eid[4][4] = {{-1, 0, 1, 2}, {0, -1, 3, 4}, {1, 3, -1, 5}, {2, 4, 5, -1}};

constexpr uint64_t KEY_NONE = ~0ull;

__device__ __forceinline__ int64_t gtid() { return nm_xcd_block() * blockDim.x + threadIdx.x; }

// element-local index of face-local node q (vertices, then edges 01,02,12)
__device__ __forceinline__ int face_local(int f, int q) {
  if (q < 3) return c_facev[f][q];
  const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
  int u = c_facev[f][pa[q - 3]], v = c_facev[f][pb[q - 3]];
  return 4 + c_eid[u][v];
}

// ---------------------------------------------------------------- geometry
// geo[t] = {dr_j/dx_i (9, [j][i]), J}; J = det(dx/dr) of the affine map from
// the reference tetrahedron (|K| = 4J/3).
__global__ void k_tet_geometry(const double* __restrict__ xyz, const int32_t* __restrict__ tet, int64_t T,
                               double* __restrict__ geo, int64_t* __restrict__ bad) {
  int64_t t = gtid();
  if (t >= T) return;
  const int32_t* v = tet + 4 * t;
  double X0[3], A[3][3];  // A columns: (X_j - X_0)/2 = dx/dr_j
  for (int c = 0; c < 3; ++c) X0[c] = xyz[3 * (int64_t)v[0] + c];
  for (int j = 0; j < 3; ++j)
    for (int c = 0; c < 3; ++c) A[c][j] = 0.5 * (xyz[3 * (int64_t)v[j + 1] + c] - X0[c]);
  double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
               A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
               A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
  double* g = geo + 10 * t;
  if (!(det > 0.0)) {
    atomicMin((unsigned long long*)bad, (unsigned long long)t);
    det = 1.0;
  }
  double id = 1.0 / det;
  // inverse of A: rows j = dr_j/dx
  g[0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) * id;
  g[1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * id;
  g[2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * id;
  g[3] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) * id;
  g[4] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * id;
  g[5] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * id;
  g[6] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) * id;
  g[7] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * id;
  g[8] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * id;
  g[9] = det;
}

// -------------------------------------------------------------- numbering
__global__ void k_edge_keys(const int32_t* __restrict__ tet, int64_t T, uint64_t* keys, uint32_t* vals) {
  int64_t i = gtid();
  if (i >= 6 * T) return;
  int64_t t = i / 6;
  int e = (int)(i % 6);
  uint64_t a = (uint32_t)tet[4 * t + c_edge[e][0]], b = (uint32_t)tet[4 * t + c_edge[e][1]];
  keys[i] = a < b ? (a << 32 | b) : (b << 32 | a);
  vals[i] = (uint32_t)i;
}

__global__ void k_head_flags(const uint64_t* __restrict__ keys, int64_t n, int32_t* flags) {
  int64_t s = gtid();
  if (s >= n) return;
  flags[s] = (s == 0 || keys[s] != keys[s - 1]) ? 1 : 0;
}

__global__ void k_geom_vertices(const int32_t* __restrict__ tet, int64_t T, int gs, int32_t* geom) {
  int64_t i = gtid();
  if (i >= 4 * T) return;
  geom[(i / 4) * gs + (i % 4)] = tet[i];
}

__global__ void k_geom_edges(const uint32_t* __restrict__ vals, const int32_t* __restrict__ seg, int64_t n,
                             int64_t V, int32_t* geom) {
  int64_t s = gtid();
  if (s >= n) return;
  uint32_t v = vals[s];
  geom[(int64_t)(v / 6) * 10 + 4 + (v % 6)] = (int32_t)(V + seg[s]);
}

__global__ void k_node_flags(const int32_t* __restrict__ geom, int gs, int64_t T, const int8_t* __restrict__ region,
                             int nd, int npp, uint32_t* flags) {
  int64_t i = gtid();
  if (i >= T * gs) return;
  int64_t t = i / gs;
  int a = (int)(i % gs);
  bool fluid = region[t] != 0;
  uint32_t bits = 0;
  if (a < nd) bits |= fluid ? 2u : 1u;
  if (fluid && a < npp) bits |= 4u;
  if (bits) atomicOr(&flags[geom[i]], bits);
}

__global__ void k_split_flags(const uint32_t* __restrict__ f, int64_t n, int32_t* s, int32_t* fl, int32_t* p) {
  int64_t i = gtid();
  if (i >= n) return;
  s[i] = f[i] & 1u;
  fl[i] = (f[i] >> 1) & 1u;
  p[i] = (f[i] >> 2) & 1u;
}

__global__ void k_elem_nodes(const int32_t* __restrict__ geom, int gs, int64_t T, const int8_t* __restrict__ region,
                             int nd, int npp, const int32_t* __restrict__ sid, const int32_t* __restrict__ fid,
                             int64_t nsolid, const int32_t* __restrict__ pid, int32_t* en, int32_t* ep) {
  int64_t t = gtid();
  if (t >= T) return;
  bool fluid = region[t] != 0;
  for (int a = 0; a < nd; ++a) {
    int32_t g = geom[t * gs + a];
    en[t * nd + a] = fluid ? (int32_t)(nsolid + fid[g]) : sid[g];
  }
  for (int c = 0; c < npp; ++c) ep[t * npp + c] = fluid ? pid[geom[t * gs + c]] : -1;
}

__global__ void k_node_geom(const uint32_t* __restrict__ f, int64_t n, const int32_t* __restrict__ sid,
                            const int32_t* __restrict__ fid, int64_t nsolid, const int32_t* __restrict__ pid,
                            int32_t* node_geom, int32_t* pres_geom) {
  int64_t g = gtid();
  if (g >= n) return;
  if (f[g] & 1u) node_geom[sid[g]] = (int32_t)g;
  if (f[g] & 2u) node_geom[nsolid + fid[g]] = (int32_t)g;
  if (f[g] & 4u) pres_geom[pid[g]] = (int32_t)g;
}

// ------------------------------------------------------ fluid-solid faces
__global__ void k_face_keys(const int32_t* __restrict__ tet, int64_t T, uint64_t* keys, uint32_t* vals) {
  int64_t i = gtid();
  if (i >= 4 * T) return;
  int64_t t = i / 4;
  int f = (int)(i % 4);
  uint64_t a = (uint32_t)tet[4 * t + c_facev[f][0]], b = (uint32_t)tet[4 * t + c_facev[f][1]],
           c = (uint32_t)tet[4 * t + c_facev[f][2]];
  uint64_t x, y, z;  // sort three
  x = a < b ? a : b; y = a < b ? b : a;
  if (c < x) { z = y; y = x; x = c; } else if (c < y) { z = y; y = c; } else { z = c; }
  keys[i] = (x << 42) | (y << 21) | z;
  vals[i] = (uint32_t)i;
}

__global__ void k_fs_flags(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals, int64_t n,
                           const int8_t* __restrict__ region, int32_t* flags) {
  int64_t s = gtid();
  if (s >= n) return;
  int fl = 0;
  if (s + 1 < n && keys[s] == keys[s + 1]) {
    int r0 = region[vals[s] / 4], r1 = region[vals[s + 1] / 4];
    fl = (r0 != r1) ? 1 : 0;
  }
  flags[s] = fl;
}

// fs[k] = {solid tet, local face of the solid tet, fluid tet}
__global__ void k_fs_compact(const uint32_t* __restrict__ vals, const int32_t* __restrict__ flags,
                             const int32_t* __restrict__ pos, int64_t n, const int8_t* __restrict__ region,
                             int32_t* fs) {
  int64_t s = gtid();
  if (s >= n || !flags[s]) return;
  uint32_t v0 = vals[s], v1 = vals[s + 1];
  bool s0 = region[v0 / 4] == 0;
  uint32_t vs = s0 ? v0 : v1, vf = s0 ? v1 : v0;
  int64_t k = pos[s];
  fs[3 * k + 0] = (int32_t)(vs / 4);
  fs[3 * k + 1] = (int32_t)(vs % 4);
  fs[3 * k + 2] = (int32_t)(vf / 4);
}

// fgeo[k] = {nu^{s->f} (3), J2D}; J2D = area / 2 (reference triangle area 2)
__global__ void k_face_geometry(const double* __restrict__ xyz, const int32_t* __restrict__ tet,
                                const int32_t* __restrict__ fs, int64_t nf, double* fgeo) {
  int64_t k = gtid();
  if (k >= nf) return;
  int64_t t = fs[3 * k];
  int f = fs[3 * k + 1];
  const int32_t* v = tet + 4 * t;
  double A[3], B[3], C[3], O[3];
  for (int c = 0; c < 3; ++c) {
    A[c] = xyz[3 * (int64_t)v[c_facev[f][0]] + c];
    B[c] = xyz[3 * (int64_t)v[c_facev[f][1]] + c];
    C[c] = xyz[3 * (int64_t)v[c_facev[f][2]] + c];
    O[c] = xyz[3 * (int64_t)v[f] + c];
  }
  double u[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]}, w[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
  double nrm[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
  double len = sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
  double s = ((A[0] - O[0]) * nrm[0] + (A[1] - O[1]) * nrm[1] + (A[2] - O[2]) * nrm[2]) < 0 ? -1.0 : 1.0;
  for (int c = 0; c < 3; ++c) fgeo[4 * k + c] = s * nrm[c] / len;
  fgeo[4 * k + 3] = 0.25 * len;  // area = len/2, J2D = area/2
}

// ------------------------------------------------------ element matrices
// Ke[(t*nd + a)*nd + b][i][j]: 3x3 block (test node a comp i, trial node b
// comp j) of the solid stiffness with gravity:
//   J (D_i)^T c_ijmn M D_m                                  (elasticity)
//   S{ J D_i^T rho M D_{g'_j} - J rho D_{d_i g'_j} M
//      - J D_j^T M rho D_{g'_i} }                           (gravity, Appendix A)
__global__ void k_elem_stiffness(int64_t T, int nd, const int8_t* __restrict__ region,
                                 const double* __restrict__ geo, const double* __restrict__ lam,
                                 const double* __restrict__ mu, const double* __restrict__ rho,
                                 const double* __restrict__ gp, const double* __restrict__ dgp, int gnp,
                                 const RefTables* __restrict__ R, double* __restrict__ Ke) {
  int64_t i = gtid();
  int64_t nn = (int64_t)nd * nd;
  if (i >= T * nn) return;
  int64_t t = i / nn;
  int a = (int)((i % nn) / nd), b = (int)(i % nd);
  double* out = Ke + 9 * i;
  if (region[t] != 0) {
    for (int q = 0; q < 9; ++q) out[q] = 0.0;
    return;
  }
  const double* g = geo + 10 * t;
  const double J = g[9];
  double rx[3][3];  // rx[j][m] = dr_j/dx_m
  for (int j = 0; j < 3; ++j)
    for (int m = 0; m < 3; ++m) rx[j][m] = g[3 * j + m];
  // S[m][n] = int d_m l_a d_n l_b = J sum_jl rx[j][m] rx[l][n] KR[j][l][a][b]
  double S[3][3];
  for (int m = 0; m < 3; ++m)
    for (int n = 0; n < 3; ++n) {
      double s = 0;
      for (int j = 0; j < 3; ++j)
        for (int l = 0; l < 3; ++l) s += rx[j][m] * rx[l][n] * R->KR[j][l][a][b];
      S[m][n] = J * s;
    }
  const double L = lam[t], U = mu[t];
  const double tr = S[0][0] + S[1][1] + S[2][2];
  double K[3][3];
  for (int p = 0; p < 3; ++p)
    for (int q = 0; q < 3; ++q) K[p][q] = L * S[p][q] + U * S[q][p] + (p == q ? U * tr : 0.0);
  if (gp) {
    // P_ac[m] = int d_m l_a l_b,  P_ca[m] = int d_m l_b l_a
    double Pab[3], Pba[3];
    for (int m = 0; m < 3; ++m) {
      double s1 = 0, s2 = 0;
      for (int j = 0; j < 3; ++j) {
        s1 += rx[j][m] * R->DR[j][a][b];
        s2 += rx[j][m] * R->DR[j][b][a];
      }
      Pab[m] = J * s1;
      Pba[m] = J * s2;
    }
    const double Mab = J * R->MM[a][b];
    const double* ga = gp + (t * gnp + a) * 3;
    const double* gb = gp + (t * gnp + b) * 3;
    const double* da = dgp + (t * gnp + a) * 9;
    const double* db = dgp + (t * gnp + b) * 9;
    const double r = rho[t];
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) {
        // G(a,p,b,q) and G(b,q,a,p), then symmetrise
        double g1 = Pab[p] * gb[q] - da[3 * p + q] * Mab - Pab[q] * gb[p];
        double g2 = Pba[q] * ga[p] - db[3 * q + p] * Mab - Pba[p] * ga[q];
        K[p][q] += 0.5 * r * (g1 + g2);
      }
  }
  for (int p = 0; p < 3; ++p)
    for (int q = 0; q < 3; ++q) out[3 * p + q] = K[p][q];
}

// Kf[(f*nfd + a)*nfd + b][i][j]: symmetrised fluid-solid face term
// S{ J2D rho^f D_{g'_i} M2 nu_j } on the solid side (Appendix A).
__global__ void k_face_gravity(int64_t nf, int nfd, const int32_t* __restrict__ fs, const double* __restrict__ fgeo,
                               const double* __restrict__ rho, const double* __restrict__ gp, int gnp,
                               const RefTables* __restrict__ R, double* __restrict__ Kf) {
  int64_t i = gtid();
  int64_t nn = (int64_t)nfd * nfd;
  if (i >= nf * nn) return;
  int64_t k = i / nn;
  int a = (int)((i % nn) / nfd), b = (int)(i % nfd);
  int64_t st = fs[3 * k], ft = fs[3 * k + 2];
  int f = fs[3 * k + 1];
  const double* nu = fgeo + 4 * k;
  const double J2 = fgeo[4 * k + 3];
  const double w = 0.5 * rho[ft] * J2 * R->M2[a][b];
  const double* ga = gp + (st * gnp + face_local(f, a)) * 3;
  const double* gb = gp + (st * gnp + face_local(f, b)) * 3;
  double* out = Kf + 9 * i;
  for (int p = 0; p < 3; ++p)
    for (int q = 0; q < 3; ++q) out[3 * p + q] = w * (ga[p] * nu[q] + gb[q] * nu[p]);
}

// ------------------------------------------------------ pattern keys
__global__ void k_graph_keys(const int32_t* __restrict__ en, int64_t T, int nd, const int32_t* __restrict__ fs,
                             int64_t nf, int nfd, uint64_t* keys, uint32_t* vals) {
  int64_t i = gtid();
  int64_t ne = T * nd * nd;
  int64_t nfc = nf * nfd * nfd;
  if (i >= ne + nfc) return;
  uint64_t r, c;
  if (i < ne) {
    int64_t t = i / (nd * nd);
    int a = (int)((i / nd) % nd), b = (int)(i % nd);
    r = (uint32_t)en[t * nd + a];
    c = (uint32_t)en[t * nd + b];
  } else {
    int64_t j = i - ne;
    int64_t k = j / (nfd * nfd);
    int a = (int)((j / nfd) % nfd), b = (int)(j % nfd);
    int64_t st = fs[3 * k];
    int f = fs[3 * k + 1];
    r = (uint32_t)en[st * nd + face_local(f, a)];
    c = (uint32_t)en[st * nd + face_local(f, b)];
  }
  keys[i] = r << 32 | c;
  vals[i] = (uint32_t)i;
}

__global__ void k_kp_keys(const int32_t* __restrict__ ep, int64_t T, int npp, const int8_t* __restrict__ region,
                          uint64_t* keys, uint32_t* vals) {
  int64_t i = gtid();
  int64_t nn = (int64_t)npp * npp;
  if (i >= T * nn) return;
  int64_t t = i / nn;
  int a = (int)((i / npp) % npp), c = (int)(i % npp);
  vals[i] = (uint32_t)i;
  if (region[t] == 0) { keys[i] = KEY_NONE; return; }
  keys[i] = ((uint64_t)(uint32_t)ep[t * npp + a]) << 32 | (uint32_t)ep[t * npp + c];
}

// E_G contributions: fluid tets (t, a, c) then fluid-solid faces (k, a, c);
// transpose = 1 swaps the key halves (pressure row, node column)
__global__ void k_eg_keys(const int32_t* __restrict__ en, const int32_t* __restrict__ ep,
                          const int32_t* __restrict__ geom, int gs, const int32_t* __restrict__ pidmap, int64_t T,
                          int nd, int npp, const int8_t* __restrict__ region, const int32_t* __restrict__ fs,
                          int64_t nf, int nfd, int nfp, int transpose, uint64_t* keys, uint32_t* vals) {
  int64_t i = gtid();
  int64_t ne = T * nd * npp, nfc = nf * nfd * nfp;
  if (i >= ne + nfc) return;
  vals[i] = (uint32_t)i;
  uint64_t r, c;
  if (i < ne) {
    int64_t t = i / (nd * npp);
    if (region[t] == 0) { keys[i] = KEY_NONE; return; }
    int a = (int)((i / npp) % nd), q = (int)(i % npp);
    r = (uint32_t)en[t * nd + a];
    c = (uint32_t)ep[t * npp + q];
  } else {
    int64_t j = i - ne;
    int64_t k = j / (nfd * nfp);
    int a = (int)((j / nfp) % nfd), q = (int)(j % nfp);
    int64_t st = fs[3 * k];
    int f = fs[3 * k + 1];
    r = (uint32_t)en[st * nd + face_local(f, a)];
    c = (uint32_t)pidmap[geom[st * gs + face_local(f, q)]];
  }
  keys[i] = transpose ? (c << 32 | r) : (r << 32 | c);
}

// ------------------------------------------------------ segmented gathers
__global__ void k_pattern(const uint64_t* __restrict__ keys, const int32_t* __restrict__ flags,
                          const int32_t* __restrict__ seg, int64_t n, int32_t* col, int32_t* row_ptr,
                          int32_t* seg_start) {
  int64_t s = gtid();
  if (s >= n || !flags[s]) return;
  int64_t u = seg[s];
  uint64_t k = keys[s];
  col[u] = (int32_t)(k & 0xffffffffu);
  seg_start[u] = (int32_t)s;
  int64_t row = (int64_t)(k >> 32);
  int64_t prow = s == 0 ? -1 : (int64_t)(keys[s - 1] >> 32);
  for (int64_t r = prow + 1; r <= row; ++r) row_ptr[r] = (int32_t)u;
}

__global__ void k_gather_ag_ms(int64_t nnzb, const int32_t* __restrict__ seg_start, const uint32_t* __restrict__ vals,
                               int64_t T, int nd, const double* __restrict__ Ke, const double* __restrict__ Kf,
                               const double* __restrict__ geo, const double* __restrict__ rho,
                               const RefTables* __restrict__ R, double* __restrict__ ag, double* __restrict__ ms) {
  int64_t u = gtid();
  if (u >= nnzb) return;
  int64_t ne = T * nd * nd;
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, m = 0.0;
  for (int64_t s = seg_start[u]; s < seg_start[u + 1]; ++s) {
    int64_t c = vals[s];
    const double* blk;
    if (c < ne) {
      int64_t t = c / (nd * nd);
      int a = (int)((c / nd) % nd), b = (int)(c % nd);
      m += rho[t] * geo[10 * t + 9] * R->MM[a][b];
      blk = Ke + 9 * c;
    } else {
      blk = Kf + 9 * (c - ne);
    }
    for (int q = 0; q < 9; ++q) acc[q] += blk[q];
  }
  for (int q = 0; q < 9; ++q) ag[9 * u + q] = acc[q];
  ms[u] = m;
}

__global__ void k_gather_kp(int64_t nnz, const int32_t* __restrict__ seg_start, const uint32_t* __restrict__ vals,
                            int npp, const double* __restrict__ geo, const double* __restrict__ lam,
                            const double* __restrict__ mu, const RefTables* __restrict__ R, double* __restrict__ kp) {
  int64_t u = gtid();
  if (u >= nnz) return;
  double acc = 0.0;
  for (int64_t s = seg_start[u]; s < seg_start[u + 1]; ++s) {
    int64_t c = vals[s];
    int64_t t = c / (npp * npp);
    int a = (int)((c / npp) % npp), q = (int)(c % npp);
    double kappa = lam[t] + 2.0 * mu[t] / 3.0;
    acc += geo[10 * t + 9] / kappa * R->Mp[a][q];
  }
  kp[u] = acc;
}

// E_G 3-vectors: fluid tet  J [ (M_fp D^p_j)_{ac} - rho kappa^{-1} g'_j(a) M_fp[a][c] ]
//                face       J2D nu_j M2sp[a][c]
__global__ void k_gather_eg(int64_t nnz, const int32_t* __restrict__ seg_start, const uint32_t* __restrict__ vals,
                            int64_t T, int nd, int npp, int nfd, int nfp, const double* __restrict__ geo,
                            const double* __restrict__ fgeo, const double* __restrict__ rho,
                            const double* __restrict__ lam, const double* __restrict__ mu,
                            const double* __restrict__ gp, int gnp, const RefTables* __restrict__ R,
                            double* __restrict__ val) {
  int64_t u = gtid();
  if (u >= nnz) return;
  int64_t ne = T * nd * npp;
  double acc[3] = {0, 0, 0};
  for (int64_t s = seg_start[u]; s < seg_start[u + 1]; ++s) {
    int64_t c = vals[s];
    if (c < ne) {
      int64_t t = c / (nd * npp);
      int a = (int)((c / npp) % nd), q = (int)(c % npp);
      const double* g = geo + 10 * t;
      const double J = g[9];
      double kappa = lam[t] + 2.0 * mu[t] / 3.0;
      double w = gp ? rho[t] / kappa * R->Mfp[a][q] : 0.0;
      for (int j = 0; j < 3; ++j) {
        double qv = 0;
        for (int l = 0; l < 3; ++l) qv += g[3 * l + j] * R->QP[l][a][q];
        double gj = gp ? gp[(t * gnp + a) * 3 + j] : 0.0;
        acc[j] += J * (qv - w * gj);
      }
    } else {
      int64_t j2 = c - ne;
      int64_t k = j2 / (nfd * nfp);
      int a = (int)((j2 / nfp) % nfd), q = (int)(j2 % nfp);
      const double* fg = fgeo + 4 * k;
      for (int j = 0; j < 3; ++j) acc[j] += fg[3] * fg[j] * R->M2sp[a][q];
    }
  }
  for (int j = 0; j < 3; ++j) val[3 * u + j] = acc[j];
}

__global__ void k_diag_inv(int64_t rows, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                           const double* __restrict__ v, double* dinv) {
  int64_t r = gtid();
  if (r >= rows) return;
  double d = 0.0;
  for (int32_t k = ptr[r]; k < ptr[r + 1]; ++k)
    if (col[k] == r) d = v[k];
  dinv[r] = 1.0 / d;
}

// ------------------------------------------------ internal node ordering
// coordinates of every displacement node (element-local node -> node id;
// all writers of a node write the same value)
__global__ void k_node_coords(const int32_t* __restrict__ en, int64_t T, int nd, const double* __restrict__ xyz,
                              const int32_t* __restrict__ tet, double* coord) {
  int64_t i = gtid();
  if (i >= T * nd) return;
  int64_t t = i / nd;
  int a = (int)(i % nd);
  const int32_t* v = tet + 4 * t;
  double x[3];
  if (a < 4) {
    for (int c = 0; c < 3; ++c) x[c] = xyz[3 * (int64_t)v[a] + c];
  } else {
    int p = c_edge[a - 4][0], q = c_edge[a - 4][1];
    for (int c = 0; c < 3; ++c) x[c] = 0.5 * (xyz[3 * (int64_t)v[p] + c] + xyz[3 * (int64_t)v[q] + c]);
  }
  int64_t node = en[i];
  for (int c = 0; c < 3; ++c) coord[3 * node + c] = x[c];
}

__device__ __forceinline__ uint64_t spread21(uint64_t x) {
  x &= 0x1fffffull;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

// Hilbert-curve index of a point of the 2^21 grid, by Skilling's transpose
// form of the curve (J. Skilling, "Programming the Hilbert curve", AIP
// Conf. Proc. 707, 2004): from the top bit down, each axis either reflects
// the lower bits of axis 0 or swaps them with its own, which turns the
// coordinates into the transposed index in Gray code; Gray decoding along
// the axes and one correction mask give the index, whose bits are then
// interleaved with axis 0 most significant.  Unlike the Z-order, the curve
// never jumps: consecutive cells are face neighbours.
__device__ uint64_t hilbert21(uint32_t x0, uint32_t x1, uint32_t x2) {
  uint32_t X[3] = {x0, x1, x2};
  for (uint32_t Q = 1u << 20; Q > 1; Q >>= 1) {
    const uint32_t P = Q - 1;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (X[i] & Q) {
        X[0] ^= P;
      } else {
        const uint32_t t = (X[0] ^ X[i]) & P;
        X[0] ^= t;
        X[i] ^= t;
      }
    }
  }
  X[1] ^= X[0];
  X[2] ^= X[1];
  uint32_t t = 0;
  for (uint32_t Q = 1u << 20; Q > 1; Q >>= 1)
    if (X[2] & Q) t ^= Q - 1;
  return (spread21(X[0] ^ t) << 2) | (spread21(X[1] ^ t) << 1) | spread21(X[2] ^ t);
}

// curve key of each node: its Hilbert index on a 2^21 grid over the bounding box
__global__ void k_curve_key(const double* __restrict__ coord, int64_t N, double x0, double y0, double z0, double inv,
                            uint64_t* key, uint32_t* val) {
  int64_t i = gtid();
  if (i >= N) return;
  const double m = 2097151.0;
  uint32_t q[3];
  const double o[3] = {x0, y0, z0};
  for (int c = 0; c < 3; ++c) {
    double u = (coord[3 * i + c] - o[c]) * inv;
    u = u < 0 ? 0 : (u > 1 ? 1 : u);
    q[c] = (uint32_t)(u * m);
  }
  key[i] = hilbert21(q[0], q[1], q[2]);
  val[i] = (uint32_t)i;
}

__global__ void k_inverse_perm(const uint32_t* __restrict__ iperm, int64_t N, int32_t* perm, int32_t* ip) {
  int64_t i = gtid();
  if (i >= N) return;
  perm[iperm[i]] = (int32_t)i;
  ip[i] = (int32_t)iperm[i];
}

__global__ void k_remap(int32_t* a, int64_t n, const int32_t* __restrict__ perm) {
  int64_t i = gtid();
  if (i < n) a[i] = perm[a[i]];
}

__global__ void k_dec(int32_t* x, int64_t n) {
  int64_t i = gtid();
  if (i < n) x[i] -= 1;
}

// ---------------------------------------------------------- host helpers
struct Segs {
  DBuf<uint64_t> keys;
  DBuf<uint32_t> vals;
  DBuf<int32_t> flags, seg;
  int64_t n = 0, nseg = 0;
};

// Stable sort of (key, contribution) pairs and segment ids of equal keys.
// Only the first n_valid sorted positions are segmented (invalid keys are
// all-ones and sort last).
Segs sort_segments(DBuf<uint64_t>& kin, DBuf<uint32_t>& vin, int64_t n, int64_t n_valid, int end_bit,
                   hipStream_t st) {
  NM_REQUIRE(n < (int64_t)1 << 31, NM_EINVAL, "too many element contributions for one sort");
  Segs s;
  s.n = n_valid;
  s.keys.alloc(std::max<int64_t>(n, 1));
  s.vals.alloc(std::max<int64_t>(n, 1));
  size_t tb = 0;
  NM_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, kin.p, s.keys.p, vin.p, s.vals.p, (int)n, 0, end_bit, st));
  DBuf<char> tmp(std::max<size_t>(tb, 1));
  NM_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, tb, kin.p, s.keys.p, vin.p, s.vals.p, (int)n, 0, end_bit, st));
  if (n_valid == 0) return s;
  s.flags.alloc(n_valid);
  s.seg.alloc(n_valid);
  hipLaunchKernelGGL(k_head_flags, dim3(grid_for(n_valid)), dim3(256), 0, st, s.keys.p, n_valid, s.flags.p);
  size_t tb2 = 0;
  NM_HIP(hipcub::DeviceScan::InclusiveSum(nullptr, tb2, s.flags.p, s.seg.p, (int)n_valid, st));
  DBuf<char> tmp2(std::max<size_t>(tb2, 1));
  NM_HIP(hipcub::DeviceScan::InclusiveSum(tmp2.p, tb2, s.flags.p, s.seg.p, (int)n_valid, st));
  int32_t last;
  NM_HIP(hipMemcpyAsync(&last, s.seg.p + n_valid - 1, 4, hipMemcpyDeviceToHost, st));
  NM_HIP(hipStreamSynchronize(st));
  s.nseg = last;
  // segment ids are 1-based after the inclusive scan; make them 0-based
  hipLaunchKernelGGL(k_dec, dim3(grid_for(n_valid)), dim3(256), 0, st, s.seg.p, n_valid);
  return s;
}

int bits_for(int64_t x) {
  int b = 1;
  while (((int64_t)1 << b) <= x) ++b;
  return b;
}

// CSR from sorted segments: row_ptr [rows+1], col [nseg], seg_start [nseg+1]
void build_csr(Segs& s, int64_t rows, DBuf<int32_t>& ptr, DBuf<int32_t>& col, DBuf<int32_t>& start,
               hipStream_t st) {
  ptr.alloc(rows + 1);
  col.alloc(std::max<int64_t>(s.nseg, 1));
  start.alloc(s.nseg + 1);
  NM_HIP(hipMemsetAsync(ptr.p, 0, (rows + 1) * 4, st));
  if (s.n)
    hipLaunchKernelGGL(k_pattern, dim3(grid_for(s.n)), dim3(256), 0, st, s.keys.p, s.flags.p, s.seg.p, s.n, col.p,
                       ptr.p, start.p);
  // rows after the last used row, and the end markers
  int32_t nseg = (int32_t)s.nseg, nn = (int32_t)s.n;
  int64_t lastrow = -1;
  if (s.n) {
    uint64_t k;
    NM_HIP(hipMemcpyAsync(&k, s.keys.p + s.n - 1, 8, hipMemcpyDeviceToHost, st));
    NM_HIP(hipStreamSynchronize(st));
    lastrow = (int64_t)(k >> 32);
  }
  std::vector<int32_t> tail(rows - lastrow, nseg);
  if (!tail.empty())
    NM_HIP(hipMemcpyAsync(ptr.p + lastrow + 1, tail.data(), tail.size() * 4, hipMemcpyHostToDevice, st));
  NM_HIP(hipMemcpyAsync(start.p + s.nseg, &nn, 4, hipMemcpyHostToDevice, st));
  NM_HIP(hipStreamSynchronize(st));
}

template <class T>
DBuf<T> upload(const T* h, size_t n, hipStream_t st) {
  DBuf<T> d(std::max<size_t>(n, 1));
  if (n) NM_HIP(hipMemcpyAsync(d.p, h, n * sizeof(T), hipMemcpyHostToDevice, st));
  return d;
}

template <class T>
T read_back(const T* d, hipStream_t st) {
  T v;
  NM_HIP(hipMemcpyAsync(&v, d, sizeof(T), hipMemcpyDeviceToHost, st));
  NM_HIP(hipStreamSynchronize(st));
  return v;
}

void excl_scan(DBuf<int32_t>& in, DBuf<int32_t>& out, int64_t n, hipStream_t st) {
  size_t tb = 0;
  NM_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, in.p, out.p, (int)n, st));
  DBuf<char> tmp(std::max<size_t>(tb, 1));
  NM_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.p, tb, in.p, out.p, (int)n, st));
}

}  // namespace

void assemble(nm_pencil* P, const nm_mesh* mesh, const nm_material* mat, hipStream_t st) {
  const int64_t V = mesh->n_vert, T = mesh->n_tet;
  NM_REQUIRE(V > 0 && T > 0, NM_EINVAL, "empty mesh");
  NM_REQUIRE(mesh->disp_order == 1 || mesh->disp_order == 2, NM_EINVAL, "disp_order must be 1 or 2");
  NM_REQUIRE(mesh->pres_order >= 1 && mesh->pres_order <= mesh->disp_order, NM_EINVAL,
             "pres_order must be 1 or 2 and <= disp_order");
  NM_REQUIRE(V < (1 << 21), NM_EINVAL, "at most 2^21 - 1 vertices supported");
  NM_REQUIRE(mesh->xyz && mesh->tet && mesh->region && mat && mat->rho && mat->lam && mat->mu, NM_EINVAL,
             "null mesh or material array");
  for (int64_t i = 0; i < 4 * T; ++i)
    if (mesh->tet[i] < 0 || mesh->tet[i] >= V)
      throw Error(NM_EBADMESH, "tetrahedron " + std::to_string(i / 4) + " has vertex index out of range");
  for (int64_t t = 0; t < T; ++t)
    if (mesh->region[t] != 0 && mesh->region[t] != 1)
      throw Error(NM_EBADMESH, "tetrahedron " + std::to_string(t) + " has region other than 0/1");
  P->V = V;
  P->T = T;
  P->disp_order = mesh->disp_order;
  P->pres_order = mesh->pres_order;
  build_ref_tables(mesh->disp_order, mesh->pres_order, P->ref);
  const int nd = P->ref.nd, npp = P->ref.npp, nfd = P->ref.nfd, nfp = P->ref.nfp;
  P->nd = nd;
  P->npp = npp;
  P->gravity = mat->gprime != nullptr;
  int gnp = mat->gprime_np;
  if (P->gravity) {
    NM_REQUIRE(mat->grad_gprime != nullptr, NM_EINVAL, "gprime given without grad_gprime");
    NM_REQUIRE(gnp >= nd, NM_EINVAL, "gprime_np smaller than the nodes of the displacement element");
  }
  const int gs = std::max(nd, npp) == 10 ? 10 : 4;  // geometric nodes per tet

  // ---- upload inputs
  auto d_xyz = upload(mesh->xyz, 3 * V, st);
  auto d_tet = upload(mesh->tet, 4 * T, st);
  auto d_reg = upload(mesh->region, T, st);
  auto d_rho = upload(mat->rho, T, st);
  auto d_lam = upload(mat->lam, T, st);
  auto d_mu = upload(mat->mu, T, st);
  DBuf<double> d_gp, d_dgp;
  if (P->gravity) {
    d_gp = upload(mat->gprime, (size_t)T * gnp * 3, st);
    d_dgp = upload(mat->grad_gprime, (size_t)T * gnp * 9, st);
  }
  DBuf<RefTables> d_ref(1);
  NM_HIP(hipMemcpyAsync(d_ref.p, &P->ref, sizeof(RefTables), hipMemcpyHostToDevice, st));

  // ---- geometry and Jacobian check
  DBuf<double> geo(10 * T);
  DBuf<int64_t> bad(1);
  int64_t big = INT64_MAX;
  NM_HIP(hipMemcpyAsync(bad.p, &big, 8, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_tet_geometry, dim3(grid_for(T)), dim3(256), 0, st, d_xyz.p, d_tet.p, T, geo.p, bad.p);
  int64_t first_bad = read_back(bad.p, st);
  if (first_bad != INT64_MAX)
    throw Error(NM_EBADMESH, "tetrahedron " + std::to_string(first_bad) + " has Jacobian <= 0");

  // ---- geometric nodes (vertices, then sorted unique edges)
  DBuf<int32_t> geom((size_t)T * gs);
  hipLaunchKernelGGL(k_geom_vertices, dim3(grid_for(4 * T)), dim3(256), 0, st, d_tet.p, T, gs, geom.p);
  int64_t n_edges = 0;
  if (gs == 10) {
    DBuf<uint64_t> k(6 * T);
    DBuf<uint32_t> v(6 * T);
    hipLaunchKernelGGL(k_edge_keys, dim3(grid_for(6 * T)), dim3(256), 0, st, d_tet.p, T, k.p, v.p);
    Segs s = sort_segments(k, v, 6 * T, 6 * T, 32 + bits_for(V), st);
    n_edges = s.nseg;
    hipLaunchKernelGGL(k_geom_edges, dim3(grid_for(s.n)), dim3(256), 0, st, s.vals.p, s.seg.p, s.n, V, geom.p);
  }
  P->n_geom = V + n_edges;
  const int64_t G = P->n_geom;

  // ---- displacement and pressure numbering
  DBuf<uint32_t> flags(G);
  NM_HIP(hipMemsetAsync(flags.p, 0, G * 4, st));
  hipLaunchKernelGGL(k_node_flags, dim3(grid_for(T * gs)), dim3(256), 0, st, geom.p, gs, T, d_reg.p, nd, npp,
                     flags.p);
  DBuf<int32_t> fs_(G), ff_(G), fp_(G), sid(G), fid(G), pid(G);
  hipLaunchKernelGGL(k_split_flags, dim3(grid_for(G)), dim3(256), 0, st, flags.p, G, fs_.p, ff_.p, fp_.p);
  excl_scan(fs_, sid, G, st);
  excl_scan(ff_, fid, G, st);
  excl_scan(fp_, pid, G, st);
  P->n_solid = read_back(sid.p + G - 1, st) + read_back(fs_.p + G - 1, st);
  int64_t n_fluid = read_back(fid.p + G - 1, st) + read_back(ff_.p + G - 1, st);
  P->n_pres = read_back(pid.p + G - 1, st) + read_back(fp_.p + G - 1, st);
  P->N = P->n_solid + n_fluid;
  const int64_t N = P->N, NP = P->n_pres;
  NM_REQUIRE(N < (1 << 30) && 3 * N < INT32_MAX, NM_EINVAL, "mesh too large for 32-bit node ids");
  DBuf<int32_t> en((size_t)T * nd), ep((size_t)T * npp);
  hipLaunchKernelGGL(k_elem_nodes, dim3(grid_for(T)), dim3(256), 0, st, geom.p, gs, T, d_reg.p, nd, npp, sid.p,
                     fid.p, P->n_solid, pid.p, en.p, ep.p);
  P->node_geom.alloc(N);
  P->pres_geom.alloc(std::max<int64_t>(NP, 1));
  hipLaunchKernelGGL(k_node_geom, dim3(grid_for(G)), dim3(256), 0, st, flags.p, G, sid.p, fid.p, P->n_solid, pid.p,
                     P->node_geom.p, P->pres_geom.p);

  // ---- internal node order: displacement nodes sorted by the Hilbert index
  // of their position (stable: the solid copy of a fluid-solid node stays
  // before its fluid copy).  Rows that are close in space are close in
  // memory, so a workgroup's gathers hit the same L2 lines, and groups of
  // consecutive rows share most of their columns (on the P2 three-layer
  // planet 4-row groups touch 6 % fewer distinct columns than in Z-order,
  // and 10 % fewer of them lie more than 4096 rows away).  Exports and all
  // vectors crossing the C ABI use the canonical numbering.
  {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t v = 0; v < V; ++v)
      for (int c = 0; c < 3; ++c) {
        lo[c] = std::min(lo[c], mesh->xyz[3 * v + c]);
        hi[c] = std::max(hi[c], mesh->xyz[3 * v + c]);
      }
    double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-300});
    DBuf<double> coord(3 * N);
    hipLaunchKernelGGL(k_node_coords, dim3(grid_for(T * nd)), dim3(256), 0, st, en.p, T, nd, d_xyz.p, d_tet.p,
                       coord.p);
    DBuf<uint64_t> k(N), ks(N);
    DBuf<uint32_t> v(N), vs(N);
    hipLaunchKernelGGL(k_curve_key, dim3(grid_for(N)), dim3(256), 0, st, coord.p, N, lo[0], lo[1], lo[2], 1.0 / ext, k.p,
                       v.p);
    size_t tb = 0;
    NM_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, k.p, ks.p, v.p, vs.p, (int)N, 0, 63, st));
    DBuf<char> tmp(std::max<size_t>(tb, 1));
    NM_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, tb, k.p, ks.p, v.p, vs.p, (int)N, 0, 63, st));
    P->perm.alloc(N);
    P->iperm.alloc(N);
    hipLaunchKernelGGL(k_inverse_perm, dim3(grid_for(N)), dim3(256), 0, st, vs.p, N, P->perm.p, P->iperm.p);
    hipLaunchKernelGGL(k_remap, dim3(grid_for(T * nd)), dim3(256), 0, st, en.p, T * nd, P->perm.p);
  }

  // ---- fluid-solid faces
  DBuf<int32_t> fs;
  DBuf<double> fgeo;
  {
    DBuf<uint64_t> k(4 * T);
    DBuf<uint32_t> v(4 * T);
    hipLaunchKernelGGL(k_face_keys, dim3(grid_for(4 * T)), dim3(256), 0, st, d_tet.p, T, k.p, v.p);
    DBuf<uint64_t> ks(4 * T);
    DBuf<uint32_t> vs(4 * T);
    size_t tb = 0;
    NM_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, k.p, ks.p, v.p, vs.p, (int)(4 * T), 0, 63, st));
    DBuf<char> tmp(std::max<size_t>(tb, 1));
    NM_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, tb, k.p, ks.p, v.p, vs.p, (int)(4 * T), 0, 63, st));
    DBuf<int32_t> fl(4 * T), pos(4 * T);
    hipLaunchKernelGGL(k_fs_flags, dim3(grid_for(4 * T)), dim3(256), 0, st, ks.p, vs.p, 4 * T, d_reg.p, fl.p);
    excl_scan(fl, pos, 4 * T, st);
    P->n_fs = read_back(pos.p + 4 * T - 1, st) + read_back(fl.p + 4 * T - 1, st);
    fs.alloc(std::max<int64_t>(3 * P->n_fs, 3));
    fgeo.alloc(std::max<int64_t>(4 * P->n_fs, 4));
    if (P->n_fs) {
      hipLaunchKernelGGL(k_fs_compact, dim3(grid_for(4 * T)), dim3(256), 0, st, vs.p, fl.p, pos.p, 4 * T, d_reg.p,
                         fs.p);
      hipLaunchKernelGGL(k_face_geometry, dim3(grid_for(P->n_fs)), dim3(256), 0, st, d_xyz.p, d_tet.p, fs.p,
                         P->n_fs, fgeo.p);
    }
  }
  const int64_t NF = P->n_fs;

  // ---- element matrices
  DBuf<double> Ke((size_t)T * nd * nd * 9);
  hipLaunchKernelGGL(k_elem_stiffness, dim3(grid_for(T * nd * nd)), dim3(256), 0, st, T, nd, d_reg.p, geo.p,
                     d_lam.p, d_mu.p, d_rho.p, P->gravity ? d_gp.p : nullptr, P->gravity ? d_dgp.p : nullptr, gnp,
                     d_ref.p, Ke.p);
  const int64_t nface_c = P->gravity ? NF : 0;  // face term exists only with gravity
  DBuf<double> Kf(std::max<int64_t>(nface_c * nfd * nfd * 9, 9));
  if (nface_c)
    hipLaunchKernelGGL(k_face_gravity, dim3(grid_for(nface_c * nfd * nfd)), dim3(256), 0, st, nface_c, nfd, fs.p,
                       fgeo.p, d_rho.p, d_gp.p, gnp, d_ref.p, Kf.p);

  // ---- node graph, A_G and M_s
  {
    int64_t nc = T * nd * nd + nface_c * nfd * nfd;
    DBuf<uint64_t> k(nc);
    DBuf<uint32_t> v(nc);
    hipLaunchKernelGGL(k_graph_keys, dim3(grid_for(nc)), dim3(256), 0, st, en.p, T, nd, fs.p, nface_c, nfd, k.p,
                       v.p);
    Segs s = sort_segments(k, v, nc, nc, 32 + bits_for(N), st);
    P->nnzb = s.nseg;
    DBuf<int32_t> start;
    build_csr(s, N, P->row_ptr, P->col, start, st);
    P->ag.alloc(9 * P->nnzb);
    P->ms.alloc(P->nnzb);
    hipLaunchKernelGGL(k_gather_ag_ms, dim3(grid_for(P->nnzb)), dim3(256), 0, st, P->nnzb, start.p, s.vals.p, T, nd,
                       Ke.p, Kf.p, geo.p, d_rho.p, d_ref.p, P->ag.p, P->ms.p);
    P->mdinv.alloc(N);
    hipLaunchKernelGGL(k_diag_inv, dim3(grid_for(N)), dim3(256), 0, st, N, P->row_ptr.p, P->col.p, P->ms.p,
                       P->mdinv.p);
  }
  build_row_groups(P, st);
  build_tiles(P, st);
  Ke.release();
  Kf.release();

  // ---- pressure mass K_p and E_G
  if (NP > 0) {
    {
      int64_t nc = T * npp * npp;
      DBuf<uint64_t> k(nc);
      DBuf<uint32_t> v(nc);
      hipLaunchKernelGGL(k_kp_keys, dim3(grid_for(nc)), dim3(256), 0, st, ep.p, T, npp, d_reg.p, k.p, v.p);
      int64_t nfl = 0;
      for (int64_t t = 0; t < T; ++t) nfl += mesh->region[t] != 0;
      Segs s = sort_segments(k, v, nc, nfl * npp * npp, 64, st);
      P->nnz_kp = s.nseg;
      DBuf<int32_t> start;
      build_csr(s, NP, P->kp_ptr, P->kp_col, start, st);
      P->kp.alloc(P->nnz_kp);
      hipLaunchKernelGGL(k_gather_kp, dim3(grid_for(P->nnz_kp)), dim3(256), 0, st, P->nnz_kp, start.p, s.vals.p,
                         npp, geo.p, d_lam.p, d_mu.p, d_ref.p, P->kp.p);
      P->kpdinv.alloc(NP);
      hipLaunchKernelGGL(k_diag_inv, dim3(grid_for(NP)), dim3(256), 0, st, NP, P->kp_ptr.p, P->kp_col.p, P->kp.p,
                         P->kpdinv.p);
    }
    int64_t nfl = 0;
    for (int64_t t = 0; t < T; ++t) nfl += mesh->region[t] != 0;
    for (int tr = 0; tr < 2; ++tr) {
      int64_t nc = T * nd * npp + NF * nfd * nfp;
      DBuf<uint64_t> k(nc);
      DBuf<uint32_t> v(nc);
      hipLaunchKernelGGL(k_eg_keys, dim3(grid_for(nc)), dim3(256), 0, st, en.p, ep.p, geom.p, gs, pid.p, T, nd, npp,
                         d_reg.p, fs.p, NF, nfd, nfp, tr, k.p, v.p);
      int64_t nvalid = nfl * nd * npp + NF * nfd * nfp;
      Segs s = sort_segments(k, v, nc, nvalid, 64, st);
      DBuf<int32_t> start;
      DBuf<int32_t>& ptr = tr ? P->egt_ptr : P->eg_ptr;
      DBuf<int32_t>& col = tr ? P->egt_col : P->eg_col;
      DBuf<double>& val = tr ? P->egt_val : P->eg_val;
      build_csr(s, tr ? NP : N, ptr, col, start, st);
      P->nnzb_eg = s.nseg;
      val.alloc(3 * std::max<int64_t>(s.nseg, 1));
      hipLaunchKernelGGL(k_gather_eg, dim3(grid_for(s.nseg)), dim3(256), 0, st, s.nseg, start.p, s.vals.p, T, nd,
                         npp, nfd, nfp, geo.p, fgeo.p, d_rho.p, d_lam.p, d_mu.p, P->gravity ? d_gp.p : nullptr,
                         gnp, d_ref.p, val.p);
    }
  }
  NM_HIP(hipStreamSynchronize(st));
  NM_HIP(hipGetLastError());
}

}  // namespace nm
