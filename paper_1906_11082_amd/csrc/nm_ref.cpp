// Reference elements of the mixed CG discretisation (Appendix A of the
// paper): nodal Lagrange bases on the reference tetrahedron
// I = {r_i >= -1, r1 + r2 + r3 <= -1} and triangle {t_i >= -1, t1 + t2 <= 0},
// built from a generalised Vandermonde matrix V_in = phi_n(r_i) of a
// polynomial basis, derivative matrices D_j = (d_j V) V^{-1}, and mass
// matrices integrated by a collapsed-coordinate Gauss rule that is exact
// for the polynomial degrees involved.
#include <cmath>
#include <algorithm>
#include <array>
#include <cstring>
#include <vector>

#include "nm_internal.h"

namespace nm {

namespace {

struct Poly {
  int dim, order;
  std::vector<std::array<int, 3>> e;  // monomial exponents
};

Poly monomials(int dim, int order) {
  Poly p{dim, order, {}};
  for (int s = 0; s <= order; ++s)
    for (int i = s; i >= 0; --i)
      for (int j = s - i; j >= 0; --j) {
        int k = s - i - j;
        if (dim == 2 && k != 0) continue;
        p.e.push_back({i, j, k});
      }
  return p;
}

double mono(const std::array<int, 3>& e, const double* r) {
  return std::pow(r[0], e[0]) * std::pow(r[1], e[1]) * std::pow(r[2], e[2]);
}
double dmono(const std::array<int, 3>& e, const double* r, int j) {
  if (e[j] == 0) return 0.0;
  std::array<int, 3> f = e;
  f[j] -= 1;
  return e[j] * mono(f, r);
}

// reference nodes: vertices, then edge midpoints in the element-local order
std::vector<std::array<double, 3>> ref_nodes(int dim, int order) {
  std::vector<std::array<double, 3>> v;
  if (dim == 3) {
    v = {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}};
    if (order == 2) {
      const int E[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
      std::vector<std::array<double, 3>> m;
      for (auto& e : E)
        m.push_back({0.5 * (v[e[0]][0] + v[e[1]][0]), 0.5 * (v[e[0]][1] + v[e[1]][1]),
                     0.5 * (v[e[0]][2] + v[e[1]][2])});
      v.insert(v.end(), m.begin(), m.end());
    }
  } else {
    v = {{-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
    if (order == 2) {
      const int E[3][2] = {{0, 1}, {0, 2}, {1, 2}};
      std::vector<std::array<double, 3>> m;
      for (auto& e : E) m.push_back({0.5 * (v[e[0]][0] + v[e[1]][0]), 0.5 * (v[e[0]][1] + v[e[1]][1]), 0});
      v.insert(v.end(), m.begin(), m.end());
    }
  }
  return v;
}

// dense inverse by Gauss-Jordan with partial pivoting (row-major n x n)
std::vector<double> inverse(std::vector<double> a, int n) {
  std::vector<double> b(n * n, 0.0);
  for (int i = 0; i < n; ++i) b[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[r * n + c]) > std::fabs(a[p * n + c])) p = r;
    for (int k = 0; k < n; ++k) {
      std::swap(a[c * n + k], a[p * n + k]);
      std::swap(b[c * n + k], b[p * n + k]);
    }
    double d = a[c * n + c];
    for (int k = 0; k < n; ++k) { a[c * n + k] /= d; b[c * n + k] /= d; }
    for (int r = 0; r < n; ++r)
      if (r != c) {
        double f = a[r * n + c];
        if (f != 0.0)
          for (int k = 0; k < n; ++k) { a[r * n + k] -= f * a[c * n + k]; b[r * n + k] -= f * b[c * n + k]; }
      }
  }
  return b;
}

// Lagrange basis of one element type: coefficient matrix Cinv (modal x nodal)
struct Lagrange {
  int dim, order, np;
  Poly P;
  std::vector<double> Cinv;  // [np][np] row-major: l_n = sum_a Cinv[a][n] phi_a
  explicit Lagrange(int d, int o) : dim(d), order(o), P(monomials(d, o)) {
    auto nodes = ref_nodes(d, o);
    np = (int)nodes.size();
    std::vector<double> Vm(np * np);
    for (int i = 0; i < np; ++i)
      for (int a = 0; a < np; ++a) Vm[i * np + a] = mono(P.e[a], nodes[i].data());
    Cinv = inverse(Vm, np);
  }
  void eval(const double* r, double* l) const {
    for (int n = 0; n < np; ++n) {
      double s = 0;
      for (int a = 0; a < np; ++a) s += Cinv[a * np + n] * mono(P.e[a], r);
      l[n] = s;
    }
  }
  void deval(const double* r, int j, double* l) const {
    for (int n = 0; n < np; ++n) {
      double s = 0;
      for (int a = 0; a < np; ++a) s += Cinv[a * np + n] * dmono(P.e[a], r, j);
      l[n] = s;
    }
  }
  // derivative matrix D_j[node i][node m] = d_j l_m (r_i)
  std::vector<double> Dmat(int j) const {
    auto nodes = ref_nodes(dim, order);
    std::vector<double> D(np * np), l(np);
    for (int i = 0; i < np; ++i) {
      deval(nodes[i].data(), j, l.data());
      for (int m = 0; m < np; ++m) D[i * np + m] = l[m];
    }
    return D;
  }
};

// Gauss-Legendre nodes/weights on [0,1] (Golub-Welsch via Jacobi eigen)
void gauss01(int n, std::vector<double>& x, std::vector<double>& w) {
  std::vector<double> J(n * n, 0.0), ev, vec;
  for (int i = 1; i < n; ++i) {
    double b = i / std::sqrt(4.0 * i * i - 1.0);
    J[i * n + i - 1] = J[(i - 1) * n + i] = b;
  }
  jacobi_eig(n, J, ev, &vec);
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    x[i] = 0.5 * (ev[i] + 1.0);
    double v0 = vec[i * n + 0];  // first component of eigenvector i (column-major)
    w[i] = v0 * v0;              // weights on [-1,1] sum to 2 -> 2 v0^2; on [0,1] halve
  }
}

struct Quad {
  std::vector<std::array<double, 3>> r;
  std::vector<double> w;
};

// collapsed (Duffy) tensor Gauss rule on the reference simplex
Quad simplex_rule(int dim, int n) {
  std::vector<double> x, w;
  gauss01(n, x, w);
  Quad q;
  if (dim == 3) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) {
          double a = x[i], b = x[j], c = x[k];
          double px = a, py = (1 - a) * b, pz = (1 - a) * (1 - b) * c;
          double wt = w[i] * w[j] * w[k] * (1 - a) * (1 - a) * (1 - b) * 8.0;
          q.r.push_back({-1 + 2 * px, -1 + 2 * py, -1 + 2 * pz});
          q.w.push_back(wt);
        }
  } else {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double a = x[i], b = x[j];
        q.r.push_back({-1 + 2 * a, -1 + 2 * (1 - a) * b, 0.0});
        q.w.push_back(w[i] * w[j] * (1 - a) * 4.0);
      }
  }
  return q;
}

std::vector<double> mass(const Lagrange& A, const Lagrange& B, const Quad& q) {
  std::vector<double> M(A.np * B.np, 0.0), la(A.np), lb(B.np);
  for (size_t s = 0; s < q.w.size(); ++s) {
    A.eval(q.r[s].data(), la.data());
    B.eval(q.r[s].data(), lb.data());
    for (int a = 0; a < A.np; ++a)
      for (int b = 0; b < B.np; ++b) M[a * B.np + b] += q.w[s] * la[a] * lb[b];
  }
  return M;
}

void mass_bounds(const std::vector<double>& M, int n, double& lo, double& hi) {
  std::vector<double> B(n * n), w;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) B[i + j * n] = M[i * n + j] / std::sqrt(M[i * n + i] * M[j * n + j]);
  jacobi_eig(n, B, w, nullptr);
  lo = w.front();
  hi = w.back();
}

}  // namespace

void jacobi_eig(int n, std::vector<double>& a, std::vector<double>& w, std::vector<double>* v) {
  std::vector<double> V(n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0, tot = 0;
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        double x = a[i + j * n] * a[i + j * n];
        tot += x;
        if (i != j) off += x;
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = a[p + q * n];
        if (apq == 0.0) continue;
        double app = a[p + p * n], aqq = a[q + q * n];
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          double akp = a[k + p * n], akq = a[k + q * n];
          a[k + p * n] = c * akp - s * akq;
          a[k + q * n] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = a[p + k * n], aqk = a[q + k * n];
          a[p + k * n] = c * apk - s * aqk;
          a[q + k * n] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[k + p * n], vkq = V[k + q * n];
          V[k + p * n] = c * vkp - s * vkq;
          V[k + q * n] = s * vkp + c * vkq;
        }
      }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return a[x + x * n] < a[y + y * n]; });
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = a[idx[i] + idx[i] * n];
  if (v) {
    v->assign(n * n, 0.0);
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) (*v)[k + j * n] = V[k + idx[j] * n];
  }
}

void build_ref_tables(int disp_order, int pres_order, RefTables& t) {
  std::memset(&t, 0, sizeof(t));
  Lagrange F(3, disp_order), Pp(3, pres_order), F2(2, disp_order), P2(2, pres_order);
  t.nd = F.np;
  t.npp = Pp.np;
  t.nfd = F2.np;
  t.nfp = P2.np;
  Quad q3 = simplex_rule(3, 6), q2 = simplex_rule(2, 6);
  auto MM = mass(F, F, q3);
  auto Mp = mass(Pp, Pp, q3);
  auto Mfp = mass(F, Pp, q3);
  auto M2 = mass(F2, F2, q2);
  auto M2sp = mass(F2, P2, q2);
  int nd = F.np, np_ = Pp.np;
  for (int a = 0; a < nd; ++a)
    for (int b = 0; b < nd; ++b) t.MM[a][b] = MM[a * nd + b];
  for (int a = 0; a < np_; ++a)
    for (int b = 0; b < np_; ++b) t.Mp[a][b] = Mp[a * np_ + b];
  for (int a = 0; a < nd; ++a)
    for (int c = 0; c < np_; ++c) t.Mfp[a][c] = Mfp[a * np_ + c];
  for (int a = 0; a < F2.np; ++a)
    for (int c = 0; c < F2.np; ++c) t.M2[a][c] = M2[a * F2.np + c];
  for (int a = 0; a < F2.np; ++a)
    for (int c = 0; c < P2.np; ++c) t.M2sp[a][c] = M2sp[a * P2.np + c];
  std::vector<double> D[3], Dp[3];
  for (int j = 0; j < 3; ++j) {
    D[j] = F.Dmat(j);
    Dp[j] = Pp.Dmat(j);
  }
  for (int j = 0; j < 3; ++j) {
    for (int a = 0; a < nd; ++a)
      for (int c = 0; c < nd; ++c) {
        double s = 0;
        for (int n = 0; n < nd; ++n) s += D[j][n * nd + a] * MM[n * nd + c];
        t.DR[j][a][c] = s;
      }
    for (int l = 0; l < 3; ++l)
      for (int a = 0; a < nd; ++a)
        for (int b = 0; b < nd; ++b) {
          double s = 0;
          for (int n = 0; n < nd; ++n)
            for (int m = 0; m < nd; ++m) s += D[j][n * nd + a] * MM[n * nd + m] * D[l][m * nd + b];
          t.KR[j][l][a][b] = s;
        }
    for (int a = 0; a < nd; ++a)
      for (int c = 0; c < np_; ++c) {
        double s = 0;
        for (int d = 0; d < np_; ++d) s += Mfp[a * np_ + d] * Dp[j][d * np_ + c];
        t.QP[j][a][c] = s;
      }
  }
  mass_bounds(MM, nd, t.m_lo, t.m_hi);
  mass_bounds(Mp, np_, t.p_lo, t.p_hi);
}

}  // namespace nm
