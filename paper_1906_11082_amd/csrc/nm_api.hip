// C ABI of the library (declared in include/nmodes.h): argument checks,
// error codes and thread-local messages around the device code.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "nm_internal.h"

namespace nm {
static thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }
}  // namespace nm



namespace {
template <class T>
std::vector<T> d2h(const T* d, size_t n) {
  std::vector<T> h(n);
  if (n) NM_HIP(hipMemcpy(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost));
  return h;
}
}  // namespace

namespace nm {
namespace {
std::mutex g_alloc_mx;
AllocHooks g_alloc;
}  // namespace

void set_alloc_hooks(const AllocHooks& h) {
  std::lock_guard<std::mutex> lk(g_alloc_mx);
  g_alloc = h;
}

void* dev_alloc(size_t bytes, AllocHooks* used) {
  AllocHooks h;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mx);
    h = g_alloc;
  }
  void* p = nullptr;
  if (h.alloc) {
    p = h.alloc(bytes, nullptr, h.ctx);
    if (!p) throw Error(NM_ENOMEM, "the allocator set by nm_set_allocator returned NULL for " +
                                       std::to_string(bytes) + " bytes");
    if (((uintptr_t)p & 255u) != 0) {
      h.free_(p, nullptr, h.ctx);
      throw Error(NM_EINVAL, "the allocator set by nm_set_allocator returned memory not aligned to 256 bytes");
    }
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    throw Error(NM_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  *used = h;
  return p;
}

void dev_free(void* p, const AllocHooks& used) noexcept {
  if (used.free_) {
    // the caller's allocator may hand the memory out again at once: no
    // kernel of any stream may still use it
    (void)hipDeviceSynchronize();
    used.free_(p, nullptr, used.ctx);
  } else {
    (void)hipFree(p);
  }
}
}  // namespace nm

static nm::ApplyCfg make_cfg(const nm_pencil* p, const nm_apply_opts* o, hipStream_t st) {
  nm::ApplyCfg c;
  double mt = (o && o->minv_tol > 0) ? o->minv_tol : 1e-12;
  double pt = (o && o->kp_tol > 0) ? o->kp_tol : 1e-13;
  c.kM = (o && o->kM > 0) ? o->kM : nm::cheb_steps(p->ref.m_lo, p->ref.m_hi, mt);
  c.kP = (o && o->kP > 0) ? o->kP : nm::cheb_steps(p->ref.p_lo, p->ref.p_hi, pt);
  c.precision = o ? o->precision : 0;
  NM_REQUIRE(c.precision == 0 || c.precision == 1, NM_EINVAL, "precision must be 0 or 1");
  NM_REQUIRE(c.kM >= 2 && c.kP >= 1, NM_EINVAL, "kM must be >= 2 and kP >= 1");
  nm::set_mass_passes(const_cast<nm_pencil*>(p), c, o ? o->mass_passes : 0, mt, (o && o->kM > 0) ? o->kM : 0, st);
  return c;
}

extern "C" {

const char* nm_last_error(void) { return nm::g_err.c_str(); }

nm_status nm_set_allocator(void* (*alloc)(size_t bytes, void* stream, void* ctx),
                           void (*free_)(void* ptr, void* stream, void* ctx), void* ctx) {
  NM_TRY({
    NM_REQUIRE((alloc == nullptr) == (free_ == nullptr), NM_EINVAL, "set both allocator functions or neither");
    nm::AllocHooks h;
    h.alloc = alloc;
    h.free_ = free_;
    h.ctx = alloc ? ctx : nullptr;
    nm::set_alloc_hooks(h);
  })
}
const char* nm_version(void) { return "nmodes 0.2 (gfx950)"; }

nm_status nm_max_block_columns(int64_t n_disp, int64_t* max_cols) {
  NM_TRY({
    NM_REQUIRE(max_cols && n_disp > 0, NM_EINVAL, "need n_disp > 0 and an output");
    *max_cols = nm::max_block_columns(n_disp);
  })
}

nm_status nm_gemm_tn(int64_t n, int32_t K, int32_t q, const double* A, int32_t lda, const double* B, int32_t ldb,
                     double* C, void* stream) {
  NM_TRY({
    NM_REQUIRE((int64_t)K * q <= 0 || (C && (n <= 0 || (A && B))), NM_EINVAL, "null matrix");
    nm::DBuf<double> ws;
    const hipStream_t st = (hipStream_t)stream;
    nm::gemm_tn(n, K, q, A, lda, B, ldb, C, ws, st);
    NM_HIP(hipStreamSynchronize(st));  // the partials are freed on return
  })
}

nm_status nm_gemm_nn(int64_t n, int32_t K, int32_t q, double alpha, const double* A, int32_t lda, const double* Cm,
                     int32_t ldc, double beta, double* D, int32_t ldd, void* stream) {
  NM_TRY({
    NM_REQUIRE(n <= 0 || q <= 0 || (D && (K <= 0 || (A && Cm))), NM_EINVAL, "null matrix");
    nm::gemm_nn(n, K, q, alpha, A, lda, Cm, ldc, beta, D, ldd, (hipStream_t)stream);
  })
}

nm_status nm_assemble(const nm_mesh* mesh, const nm_material* mat, const double omega[3], void* stream,
                      nm_pencil** out) {
  NM_TRY({
    NM_REQUIRE(mesh && mat && out, NM_EINVAL, "null argument");
    *out = nullptr;
    nm_pencil* P = new nm_pencil();
    try {
      NM_HIP(hipGetDevice(&P->device));
      if (omega)
        for (int i = 0; i < 3; ++i) P->omega[i] = omega[i];
      NM_BLAS(rocblas_create_handle(&P->blas));
      nm::assemble(P, mesh, mat, (hipStream_t)stream);
    } catch (...) {
      nm_pencil_free(P);
      throw;
    }
    *out = P;
  })
}

void nm_pencil_free(nm_pencil* p) {
  if (!p) return;
  if (p->blas) rocblas_destroy_handle(p->blas);
  delete p;
}

nm_status nm_pencil_info_get(const nm_pencil* p, nm_pencil_info* info) {
  NM_TRY({
    NM_REQUIRE(p && info, NM_EINVAL, "null argument");
    info->n_geom = p->n_geom;
    info->n_node = p->N;
    info->n_solid = p->n_solid;
    info->n_disp = 3 * p->N;
    info->n_pres = p->n_pres;
    info->nnzb = p->nnzb;
    info->nnz_kp = p->nnz_kp;
    info->nnzb_eg = p->nnzb_eg;
    info->n_fs_faces = p->n_fs;
    info->minv_lo = p->ref.m_lo;
    info->minv_hi = p->ref.m_hi;
    info->kp_lo = p->ref.p_lo;
    info->kp_hi = p->ref.p_hi;
  })
}


nm_status nm_pencil_export_csr(const nm_pencil* p, int32_t which, int64_t* nrows, int64_t* ncols, int64_t* nnz,
                               int64_t* row_ptr, int32_t* col, double* val) {
  NM_TRY({
    NM_REQUIRE(p && nrows && ncols && nnz, NM_EINVAL, "null argument");
    const int64_t N = p->N, n = 3 * N, NP = p->n_pres;
    switch (which) {
      case NM_MAT_AG: case NM_MAT_R: *nrows = n; *ncols = n; *nnz = 9 * p->nnzb; break;
      case NM_MAT_M: *nrows = N; *ncols = N; *nnz = p->nnzb; break;
      case NM_MAT_KP: *nrows = NP; *ncols = NP; *nnz = p->nnz_kp; break;
      case NM_MAT_EG: *nrows = n; *ncols = NP; *nnz = NP ? 3 * p->nnzb_eg : 0; break;
      default: throw nm::Error(NM_EINVAL, "unknown matrix id");
    }
    if (!row_ptr) return NM_OK;
    NM_REQUIRE(col, NM_EINVAL, "col buffer missing");
    if (which == NM_MAT_KP) {
      if (NP == 0) { row_ptr[0] = 0; return NM_OK; }
      auto rp = d2h(p->kp_ptr.p, NP + 1);
      auto c = d2h(p->kp_col.p, *nnz);
      for (int64_t i = 0; i <= NP; ++i) row_ptr[i] = rp[i];
      std::memcpy(col, c.data(), 4 * c.size());
      if (val) {
        auto v = d2h(p->kp.p, *nnz);
        std::memcpy(val, v.data(), 8 * v.size());
      }
      return NM_OK;
    }
    // displacement rows are stored in the internal (Hilbert) node order:
    // canonical row c is internal row perm[c], internal column j is
    // canonical column iperm[j]; entries are re-sorted by canonical column
    auto perm = d2h(p->perm.p, N);
    auto iperm = d2h(p->iperm.p, N);
    if (which == NM_MAT_EG) {
      if (NP == 0) { for (int64_t i = 0; i <= n; ++i) row_ptr[i] = 0; return NM_OK; }
      auto rp = d2h(p->eg_ptr.p, N + 1);
      auto c = d2h(p->eg_col.p, p->nnzb_eg);
      std::vector<double> v;
      if (val) v = d2h(p->eg_val.p, 3 * p->nnzb_eg);
      int64_t q = 0;
      row_ptr[0] = 0;
      for (int64_t cr = 0; cr < N; ++cr) {
        const int64_t i = perm[cr];
        for (int cc = 0; cc < 3; ++cc) {
          for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {  // pressure columns are canonical and sorted
            col[q] = c[k];
            if (val) val[q] = v[3 * (int64_t)k + cc];
            ++q;
          }
          row_ptr[3 * cr + cc + 1] = q;
        }
      }
      return NM_OK;
    }
    auto rp = d2h(p->row_ptr.p, N + 1);
    auto c = d2h(p->col.p, p->nnzb);
    std::vector<double> v;
    const bool ag = which == NM_MAT_AG;
    if (val) v = d2h(ag ? p->ag.p : p->ms.p, ag ? 9 * p->nnzb : p->nnzb);
    const double* om = p->omega;
    const double Ox[3][3] = {{0, -om[2], om[1]}, {om[2], 0, -om[0]}, {-om[1], om[0], 0}};
    std::vector<std::pair<int32_t, int32_t>> ent;  // (canonical col, internal entry)
    int64_t q = 0;
    row_ptr[0] = 0;
    for (int64_t cr = 0; cr < N; ++cr) {
      const int64_t i = perm[cr];
      ent.clear();
      for (int32_t k = rp[i]; k < rp[i + 1]; ++k) ent.emplace_back(iperm[c[k]], k);
      std::sort(ent.begin(), ent.end());
      if (which == NM_MAT_M) {
        for (auto& pr : ent) {
          col[q] = pr.first;
          if (val) val[q] = v[pr.second];
          ++q;
        }
        row_ptr[cr + 1] = q;
        continue;
      }
      for (int cc = 0; cc < 3; ++cc) {
        for (auto& pr : ent)
          for (int d = 0; d < 3; ++d) {
            col[q] = 3 * pr.first + d;
            if (val) val[q] = ag ? v[9 * (int64_t)pr.second + 3 * cc + d] : v[pr.second] * Ox[cc][d];
            ++q;
          }
        row_ptr[3 * cr + cc + 1] = q;
      }
    }
  })
}

nm_status nm_pencil_nodes(const nm_pencil* p, int64_t* node_geom, int64_t* pres_geom) {
  NM_TRY({
    NM_REQUIRE(p, NM_EINVAL, "null pencil");
    if (node_geom) {
      auto h = d2h(p->node_geom.p, p->N);
      for (int64_t i = 0; i < p->N; ++i) node_geom[i] = h[i];
    }
    if (pres_geom && p->n_pres) {
      auto h = d2h(p->pres_geom.p, p->n_pres);
      for (int64_t i = 0; i < p->n_pres; ++i) pres_geom[i] = h[i];
    }
  })
}


nm_status nm_pencil_apply(const nm_pencil* p, int32_t op, int32_t ncols, const void* X, void* Y,
                          const nm_apply_opts* opts, void* stream) {
  NM_TRY({
    NM_REQUIRE(p && X && Y && X != Y, NM_EINVAL, "invalid pointers");
    nm::check_block(3 * p->N, ncols);
    nm::api_apply(p, op, ncols, X, Y, make_cfg(p, opts, (hipStream_t)stream), (hipStream_t)stream);
  })
}

nm_status nm_pencil_autotune(nm_pencil* p, int32_t precision, void* stream, int32_t* block, double* us_per_column) {
  NM_TRY({
    NM_REQUIRE(p && (precision == 0 || precision == 1), NM_EINVAL, "invalid arguments");
    int b = 0;
    double us = 0;
    nm::autotune(p, precision, (hipStream_t)stream, &b, &us);
    if (block) *block = b;
    if (us_per_column) *us_per_column = us;
  })
}

nm_status nm_filter_coeffs(double a, double b, double lmin, double lmax, int32_t m, double* mu) {
  NM_TRY({
    NM_REQUIRE(mu && m >= 0 && lmax > lmin && b > a, NM_EINVAL, "invalid filter arguments");
    nm::jackson_chebyshev(a, b, lmin, lmax, m, mu);
  })
}

nm_status nm_filter_degree(double a, double b, double lmin, double lmax, double guard, int32_t null_filter,
                           int32_t* m) {
  NM_TRY({
    NM_REQUIRE(m && lmax > lmin && b > a, NM_EINVAL, "invalid filter arguments");
    NM_REQUIRE(null_filter >= 0 && null_filter <= 3, NM_EINVAL, "mode must be 0, 1, 2 or 3");
    *m = nm::choose_degree(a, b, lmin, lmax, guard, null_filter);
  })
}

nm_status nm_filter_apply(const nm_pencil* p, const double* mu, int32_t m, double c, double e, double null_shift,
                          double null_scale, int32_t ncols, const void* X, void* Y, const nm_apply_opts* opts,
                          void* stream) {
  NM_TRY({
    NM_REQUIRE(p && mu && X && Y && X != Y && m >= 0 && e > 0 && ncols > 0, NM_EINVAL, "invalid filter arguments");
    nm::check_block(3 * p->N, ncols);
    hipStream_t st = (hipStream_t)stream;
    auto cfg = make_cfg(p, opts, st);
    // vectors cross the ABI in canonical node order; the filter runs in the internal order
    const int eb = cfg.precision == 1 ? 4 : 8;
    const int64_t w = 3 * (int64_t)ncols;
    nm::DBuf<char> xi((size_t)p->N * w * eb), yi((size_t)p->N * w * eb);
    nm::permute_rows(p->N, (int)w, X, xi.p, p->iperm.p, eb, st);
    if (cfg.precision == 1) {
      const_cast<nm_pencil*>(p)->ensure_fp32(st);
      nm::FilterWork<float> wk;
      nm::filter_apply<float>(p, mu, m, c, e, null_shift, null_scale, ncols, (const float*)xi.p, (float*)yi.p, cfg,
                              wk, st);
    } else {
      nm::FilterWork<double> wk;
      nm::filter_apply<double>(p, mu, m, c, e, null_shift, null_scale, ncols, (const double*)xi.p, (double*)yi.p,
                               cfg, wk, st);
    }
    nm::permute_rows(p->N, (int)w, yi.p, Y, p->perm.p, eb, st);
    NM_HIP(hipStreamSynchronize(st));
    NM_HIP(hipGetLastError());
  })
}

static nm_status spectrum_dos_impl(const nm_pencil* p, double lmin, double lmax, int32_t m, int32_t nvec,
                                   const double* Z, const nm_apply_opts* opts, void* stream, double* tau,
                                   bool weighted) {
  NM_TRY({
    NM_REQUIRE(p && Z && tau && m >= 0 && nvec >= 1 && lmax > lmin, NM_EINVAL, "invalid density-of-states arguments");
    nm::check_block(3 * p->N, nvec);
    hipStream_t st = (hipStream_t)stream;
    auto cfg = make_cfg(p, opts, st);
    NM_REQUIRE(cfg.precision == 0, NM_EINVAL, "the density of states runs in FP64 (precision 0)");
    const int64_t w = 3 * (int64_t)nvec;
    nm::DBuf<double> zi((size_t)p->N * w);
    nm::permute_rows(p->N, (int)w, Z, zi.p, p->iperm.p, 8, st);
    nm::dos_traces(p, lmin, lmax, m, nvec, zi.p, cfg, st, tau, weighted);
    NM_HIP(hipGetLastError());
  })
}

nm_status nm_spectrum_dos(const nm_pencil* p, double lmin, double lmax, int32_t m, int32_t nvec, const double* Z,
                          const nm_apply_opts* opts, void* stream, double* tau) {
  return spectrum_dos_impl(p, lmin, lmax, m, nvec, Z, opts, stream, tau, false);
}

nm_status nm_spectrum_dos_weighted(const nm_pencil* p, double lmin, double lmax, int32_t m, int32_t nvec,
                                   const double* Z, const nm_apply_opts* opts, void* stream, double* tau) {
  return spectrum_dos_impl(p, lmin, lmax, m, nvec, Z, opts, stream, tau, true);
}

namespace {

// n-point Gauss-Legendre rule on [-1, 1] (Newton on the three-term
// recurrence of the Legendre polynomials from the usual cosine guesses)
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Jackson-damped Chebyshev coefficients on [lmin, lmax] of f(l) = 1/l on
// [a, b] (0 elsewhere, a > 0): with l = c + e cos(th),
// c_k = (2/pi) int over [th_b, th_a] of cos(k th) / (c + e cos th) d th (c_0
// halved), by 16-point Gauss-Legendre panels short enough for cos(k th)
void inv_window_coeffs(double a, double b, double lmin, double lmax, int m, double* mu) {
  const double c = 0.5 * (lmax + lmin), e = 0.5 * (lmax - lmin);
  const double tha = std::acos(std::min(1.0, std::max(-1.0, (a - c) / e)));
  const double thb = std::acos(std::min(1.0, std::max(-1.0, (b - c) / e)));
  std::vector<double> gx, gw;
  gauss_legendre(16, gx, gw);
  const int panels = std::max(2, (int)std::ceil((m + 1) * (tha - thb) / 2.0) + 2);
  const double h = (tha - thb) / panels;
  std::vector<double> acc(m + 1, 0.0);
  for (int q = 0; q < panels; ++q) {
    for (int g = 0; g < 16; ++g) {
      const double th = thb + h * (q + 0.5 * (gx[g] + 1.0));
      const double wt = 0.5 * h * gw[g] / (c + e * std::cos(th));
      for (int k = 0; k <= m; ++k) acc[k] += wt * std::cos(k * th);
    }
  }
  const double tj = M_PI / (m + 2);
  for (int k = 0; k <= m; ++k) {
    const double jac = ((1.0 - (double)k / (m + 2)) * std::sin(tj) * std::cos(k * tj) +
                        std::cos(tj) * std::sin(k * tj) / (m + 2)) / std::sin(tj);
    mu[k] = (k == 0 ? 1.0 : 2.0) / M_PI * acc[k] * jac;
  }
}

double dos_estimate(const double* tau, int m, double lmin, double lmax, double a, double b, bool weighted,
                    std::vector<double>& mu) {
  mu.resize(m + 1);
  if (weighted)
    inv_window_coeffs(a, b, lmin, lmax, m, mu.data());
  else
    nm::jackson_chebyshev(a, b, lmin, lmax, m, mu.data());
  double s = 0;
  for (int k = 0; k <= m; ++k) s += mu[k] * tau[k];
  return s;
}

nm_status dos_count_impl(const double* tau, int32_t m, double lmin, double lmax, double a, double b, double* count,
                         bool weighted) {
  NM_TRY({
    NM_REQUIRE(tau && count && m >= 0 && lmax > lmin && b > a, NM_EINVAL, "invalid count arguments");
    NM_REQUIRE(!weighted || a > 0, NM_EINVAL, "weighted counts need a window above 0");
    std::vector<double> mu;
    *count = dos_estimate(tau, m, lmin, lmax, a, b, weighted, mu);
  })
}

nm_status dos_slices_impl(const double* tau, int32_t m, double lmin, double lmax, double a, double b,
                          int32_t nslices, double* edges, bool weighted) {
  NM_TRY({
    NM_REQUIRE(tau && edges && m >= 0 && lmax > lmin && b > a && nslices >= 1, NM_EINVAL, "invalid slice arguments");
    NM_REQUIRE(!weighted || a > 0, NM_EINVAL, "weighted counts need a window above 0");
    std::vector<double> mu;
    auto count = [&](double x) { return dos_estimate(tau, m, lmin, lmax, a, x, weighted, mu); };
    const double total = count(b);
    edges[0] = a;
    for (int i = 1; i < nslices; ++i) {
      const double target = total * i / nslices;
      double lo = edges[i - 1], hi = b;
      for (int it = 0; it < 60; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (count(mid) < target) lo = mid;
        else hi = mid;
      }
      edges[i] = 0.5 * (lo + hi);
    }
    edges[nslices] = b;
  })
}

}  // namespace

nm_status nm_dos_count(const double* tau, int32_t m, double lmin, double lmax, double a, double b, double* count) {
  return dos_count_impl(tau, m, lmin, lmax, a, b, count, false);
}

nm_status nm_dos_count_weighted(const double* tau, int32_t m, double lmin, double lmax, double a, double b,
                                double* count) {
  return dos_count_impl(tau, m, lmin, lmax, a, b, count, true);
}

nm_status nm_dos_slices(const double* tau, int32_t m, double lmin, double lmax, double a, double b, int32_t nslices,
                        double* edges) {
  return dos_slices_impl(tau, m, lmin, lmax, a, b, nslices, edges, false);
}

nm_status nm_dos_slices_weighted(const double* tau, int32_t m, double lmin, double lmax, double a, double b,
                                 int32_t nslices, double* edges) {
  return dos_slices_impl(tau, m, lmin, lmax, a, b, nslices, edges, true);
}

nm_status nm_spectrum_bound_rigorous(const nm_pencil* p, void* stream, double* lmax) {
  NM_TRY({
    NM_REQUIRE(p && lmax, NM_EINVAL, "invalid arguments");
    *lmax = nm::lmax_rigorous(p, (hipStream_t)stream);
  })
}

nm_status nm_spectrum_bounds(const nm_pencil* p, int32_t steps, uint64_t seed, void* stream, double* lmin,
                             double* lmax) {
  NM_TRY({
    NM_REQUIRE(p && lmin && lmax && steps >= 2, NM_EINVAL, "invalid arguments");
    nm::spectrum_bounds(p, steps, seed, (hipStream_t)stream, lmin, lmax);
  })
}

nm_status nm_filtered_eig(const nm_pencil* p, double a, double b, int32_t nev, double tol, const nm_eig_opts* opts,
                          nm_eig_result** out) {
  NM_TRY({
    NM_REQUIRE(p && out, NM_EINVAL, "null argument");
    *out = nullptr;
    nm_eig_opts o;
    if (opts) o = *opts;
    else {
      std::memset(&o, 0, sizeof(o));
      o.null_filter = -1;
    }
    nm::filtered_eig(p, a, b, nev, tol, o, out);
  })
}

nm_status nm_filtered_eig_slices(const nm_pencil* p, int32_t nslices, const double* a, const double* b,
                                 const int32_t* nev, double tol, const nm_eig_opts* opts, nm_eig_result** out) {
  NM_TRY({
    NM_REQUIRE(p && a && b && nev && out && nslices >= 1 && nslices <= 64, NM_EINVAL, "invalid arguments");
    for (int i = 0; i < nslices; ++i) out[i] = nullptr;
    nm_eig_opts o;
    if (opts) o = *opts;
    else {
      std::memset(&o, 0, sizeof(o));
      o.null_filter = -1;
    }
    std::vector<int> nv(nev, nev + nslices);
    nm::filtered_eig_slices(p, nslices, a, b, nv.data(), tol, o, out);
  })
}

nm_status nm_project_rotation(const nm_pencil* p, const nm_eig_result* basis, double a, double b, void* stream,
                              nm_rot_result** out) {
  NM_TRY({
    NM_REQUIRE(p && basis && out && b > a, NM_EINVAL, "invalid arguments");
    *out = nullptr;
    nm::project_rotation(p, basis, a, b, (hipStream_t)stream, out);
  })
}

nm_status nm_refine_rotation(const nm_pencil* p, const nm_eig_result* basis, const nm_rot_result* rot, double a,
                             double b, int32_t iters, int32_t degree, double tol, void* stream, nm_rot_result** out) {
  NM_TRY({
    NM_REQUIRE(p && basis && rot && out && b > a, NM_EINVAL, "invalid arguments");
    *out = nullptr;
    nm::refine_rotation(p, basis, rot, a, b, iters, degree, tol, (hipStream_t)stream, out);
  })
}

nm_status nm_result_copy_vectors(const nm_eig_result* r, void* dst, int32_t dst_is_device) {
  NM_TRY({
    NM_REQUIRE(r && dst, NM_EINVAL, "null argument");
    if (r->count)
      NM_HIP(hipMemcpy(dst, r->X, 8 * (size_t)r->n * r->count,
                       dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
  })
}

nm_status nm_rot_copy_vectors(const nm_rot_result* r, void* dst, int32_t dst_is_device) {
  NM_TRY({
    NM_REQUIRE(r && dst, NM_EINVAL, "null argument");
    if (r->count)
      NM_HIP(hipMemcpy(dst, r->U, 16 * (size_t)r->n * r->count,
                       dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
  })
}

void nm_result_free(nm_eig_result* r) {
  if (!r) return;
  if (r->X) (void)hipFree(r->X);
  std::free(r->lambda);
  std::free(r->resid);
  delete r;
}

void nm_rot_result_free(nm_rot_result* r) {
  if (!r) return;
  if (r->U) (void)hipFree(r->U);
  std::free(r->omega);
  std::free(r->resid);
  std::free(r);
}

}  // extern "C"
