// Several spectral windows of one pencil solved together (spectrum slicing,
// Sec. 6.1 cites it; here the slices share every filter application): one
// host thread and stream per slice runs the block Lanczos of that slice, and
// their filter applications are concatenated column-wise into one block with
// one Chebyshev series per column, so the sparse products stream the
// matrices once for all slices.  The recurrence of the filter is the same for
// every column (all slices use the interval [c - e, c + e]); a column's
// result depends only on its own series, so a slice's result is the same
// batched or alone.
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cstring>
#include <thread>

#include "nm_internal.h"

namespace nm {

FilterBatcher::FilterBatcher(const nm_pencil* P, int precision, const ApplyCfg& cfg, double c, double e, int active,
                             hipStream_t st)
    : P_(P), prec_(precision), cfg_(cfg), c_(c), e_(e), active_(active), st_(st) {
  cfg_.prof = &prof;
}

int FilterBatcher::filter(const double* X, double* Y, const double* mu, int m, int bs) {
  Req r{X, Y, mu, m, bs, 0, false, nullptr};
  std::unique_lock<std::mutex> lk(mx_);
  pend_.push_back(&r);
  if ((int)pend_.size() == active_) run_locked();
  cv_.wait(lk, [&] { return r.done; });
  if (r.err) std::rethrow_exception(r.err);
  return r.deg;
}

void FilterBatcher::leave() {
  std::unique_lock<std::mutex> lk(mx_);
  --active_;
  if (active_ > 0 && (int)pend_.size() == active_) run_locked();
}

void FilterBatcher::run_locked() {
  std::vector<Req*> batch;
  batch.swap(pend_);
  try {
    const int64_t n = 3 * P_->N;
    int ct = 0, mmax = 1;
    for (Req* q : batch) {
      ct += q->bs;
      mmax = std::max(mmax, q->m);
    }
    check_block(n, ct);
    // per-column series, zero-padded to the largest degree
    std::vector<double> mu((size_t)(mmax + 1) * ct, 0.0);
    int o = 0;
    for (Req* q : batch) {
      for (int k = 0; k <= q->m; ++k)
        for (int j = 0; j < q->bs; ++j) mu[(size_t)k * ct + o + j] = q->mu[k];
      o += q->bs;
    }
    if (xb_.n < (size_t)n * ct) {
      xb_.alloc((size_t)n * ct);
      yb_.alloc((size_t)n * ct);
      if (prec_) {
        x32_.alloc((size_t)n * ct);
        y32_.alloc((size_t)n * ct);
      }
    }
    o = 0;
    for (Req* q : batch) {
      NM_HIP(hipMemcpy2DAsync(xb_.p + o, 8 * (size_t)ct, q->X, 8 * (size_t)q->bs, 8 * (size_t)q->bs, n,
                              hipMemcpyDeviceToDevice, st_));
      o += q->bs;
    }
    if (prec_ == 0) {
      filter_apply_cols<double>(P_, mu.data(), mmax, c_, e_, ct, xb_.p, yb_.p, cfg_, fw_, st_);
    } else {
      convert_f64_f32(n * ct, xb_.p, x32_.p, st_);
      filter_apply_cols<float>(P_, mu.data(), mmax, c_, e_, ct, x32_.p, y32_.p, cfg_, fw32_, st_);
      convert_f32_f64(n * ct, y32_.p, yb_.p, st_);
    }
    o = 0;
    for (Req* q : batch) {
      NM_HIP(hipMemcpy2DAsync(q->Y, 8 * (size_t)q->bs, yb_.p + o, 8 * (size_t)ct, 8 * (size_t)q->bs, n,
                              hipMemcpyDeviceToDevice, st_));
      o += q->bs;
    }
    NM_HIP(hipStreamSynchronize(st_));
    for (Req* q : batch) q->deg = mmax;
  } catch (...) {
    for (Req* q : batch) q->err = std::current_exception();
  }
  for (Req* q : batch) q->done = true;
  cv_.notify_all();
}

void filtered_eig_slices(const nm_pencil* P, int S, const double* a, const double* b, const int* nev, double tol,
                         const nm_eig_opts& o, nm_eig_result** out) {
  NM_REQUIRE(S >= 1 && a && b && nev && out && tol > 0, NM_EINVAL, "invalid slice arguments");
  for (int i = 0; i < S; ++i) {
    out[i] = nullptr;
    NM_REQUIRE(b[i] > a[i] && nev[i] > 0, NM_EINVAL, "every slice needs a < b and nev > 0");
  }
  NM_REQUIRE(o.null_filter != 1, NM_EINVAL, "batched slices do not take the null factor");
  NM_REQUIRE(o.precision == 0 || o.precision == 1, NM_EINVAL, "precision must be 0 or 1");
  {
    // the batched filter block concatenates every window's block
    int64_t width = 0;
    for (int i = 0; i < S; ++i) width += solve_block_width(P, o, nev[i]);
    check_block(3 * P->N, width);
  }
  hipStream_t st = (hipStream_t)o.stream;
  int dev = 0;
  NM_HIP(hipGetDevice(&dev));
  if (o.precision == 1) const_cast<nm_pencil*>(P)->ensure_fp32(st);
  // common filter interval
  double lmin = o.lmin, lmax = o.lmax;
  if (!(lmax > lmin)) {
    spectrum_bounds(P, 60, o.seed ^ 0x5bd1e995ull, st, &lmin, &lmax);
    double wmax = 0;
    for (int i = 0; i < S; ++i) wmax = std::max(wmax, b[i] - a[i]);
    lmin -= 1e-3 * wmax;
  }
  // the inner-solve configuration every slice would choose (filtered_eig's defaults)
  ApplyCfg cfg;
  const int prec = o.precision;
  const double mtol = o.minv_tol > 0 ? o.minv_tol : (prec ? 1e-7 : std::min(1e-7, std::max(1e-12, 0.3 * tol)));
  const double ptol = o.kp_tol > 0 ? o.kp_tol : (prec ? 1e-7 : 1e-13);
  cfg.kM = cheb_steps(P->ref.m_lo, P->ref.m_hi, mtol);
  cfg.kP = cheb_steps(P->ref.p_lo, P->ref.p_hi, ptol);
  cfg.precision = prec;
  // before the slice threads start: creates the FP32 shadows the mixed solve reads
  set_mass_passes(const_cast<nm_pencil*>(P), cfg, o.mass_passes, mtol, 0, st);
  FilterBatcher fb(P, prec, cfg, 0.5 * (lmax + lmin), 0.5 * (lmax - lmin), S, st);

  std::vector<std::exception_ptr> errs(S);
  std::vector<int> codes(S, NM_OK);
  std::vector<std::thread> th;
  for (int i = 0; i < S; ++i) {
    th.emplace_back([&, i]() {
      hipStream_t ss = nullptr;
      rocblas_handle h = nullptr;
      BatchSeat seat{&fb};
      try {
        NM_HIP(hipSetDevice(dev));
        NM_HIP(hipStreamCreateWithFlags(&ss, hipStreamNonBlocking));
        NM_BLAS(rocblas_create_handle(&h));
        nm_eig_opts oi = o;
        oi.lmin = lmin;
        oi.lmax = lmax;
        oi.stream = ss;
        oi.seed = o.seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
        filtered_eig(P, a[i], b[i], nev[i], tol, oi, &out[i], &seat, h);
      } catch (const Error& e) {
        codes[i] = e.code;
        if (e.code != NM_PARTIAL) errs[i] = std::current_exception();
      } catch (...) {
        codes[i] = NM_EDEVICE;
        errs[i] = std::current_exception();
      }
      seat.leave();
      if (h) rocblas_destroy_handle(h);
      if (ss) (void)hipStreamDestroy(ss);
    });
  }
  for (auto& t : th) t.join();
  // hot-kernel statistics of the batched applications
  fb.prof.harvest();
  int ctot = 0;
  for (int i = 0; i < S; ++i)
    if (out[i]) ctot += out[i]->block;
  for (int i = 0; i < S; ++i) {
    if (!out[i]) continue;
    out[i]->hot_launches = fb.prof.launches;
    out[i]->hot_samples = fb.prof.samples;
    out[i]->hot_ms = fb.prof.samples ? fb.prof.ms / fb.prof.samples : 0.0;
    const double sz = (prec || cfg.mixP) ? 4.0 : 8.0;
    out[i]->hot_bytes = (double)P->nnzb * (4.0 + sz) + 4.0 * (P->N + 1) + sz * P->N + 4.0 * 3 * P->N * ctot * sz;
    out[i]->hot_kernel = mass_kernel_kind(P, ctot, prec == 1 || cfg.mixP > 0);
  }
  for (int i = 0; i < S; ++i)
    if (errs[i]) {
      for (int k = 0; k < S; ++k) {
        nm_result_free(out[k]);
        out[k] = nullptr;
      }
      std::rethrow_exception(errs[i]);
    }
  for (int i = 0; i < S; ++i)
    if (codes[i] == NM_PARTIAL) throw Error(NM_PARTIAL, "a slice did not converge all pairs in its window");
}

}  // namespace nm
