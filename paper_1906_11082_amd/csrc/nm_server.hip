// Request server: solves of different planets and windows submitted at any
// time, admitted in arrival order while the sum of their estimated device
// memory stays within a budget (and at most max_active run at once), each run
// on its own host thread and HIP stream so that admitted requests overlap on
// the device; the pencil (matrices) stays resident for the whole request,
// whose windows share filter applications (nm_filtered_eig_slices).
// Results are what the same request gives alone: every computation of a
// request depends only on its own inputs.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <thread>

#include "nm_internal.h"

namespace {

using clk = std::chrono::steady_clock;

struct Job {
  int64_t id = 0;
  // copies of the request (the caller's arrays are borrowed only during submit)
  std::vector<double> xyz, rho, lam, mu, gp, dgp, a, b;
  std::vector<int32_t> tet, nev;
  std::vector<int8_t> region;
  nm_mesh mesh{};
  nm_material mat{};
  double omega[3] = {0, 0, 0};
  double tol = 1e-8;
  nm_eig_opts opts{};
  int32_t rotate = 0;
  double est = 0;
  // outcome
  bool done = false;
  nm_server_result* res = nullptr;
  std::thread th;
};

}  // namespace

struct nm_server {
  double budget = 0;
  int max_active = 1;
  int device = 0;
  clk::time_point t0 = clk::now();
  std::mutex mx;
  std::condition_variable cv;
  std::deque<Job*> queue;
  std::map<int64_t, Job*> jobs;
  int64_t next_id = 1;
  double in_use = 0;
  int active = 0;
  bool stopping = false;
  std::thread sched;

  double now() const { return std::chrono::duration<double>(clk::now() - t0).count(); }
};

namespace nm {

// Device memory estimate of a request (bytes), from the mesh sizes before
// assembly: node count N ~ V (P1) or 2V + T (P2, edges ~ V + T); node-graph
// blocks ~ 15 N (P1) or 28 N (P2); matrices (A_G 3x3 blocks, M_s, indices,
// row-group coefficients, FP32 shadows), element-matrix staging of the
// assembly, and per window the Krylov basis and A times it (K = max(6 nev,
// nev + 16 b, 320) columns each), the filter workspace and the refinement.
double request_bytes(const nm_mesh& m, int S, const int32_t* nev, const nm_eig_opts& o) {
  const double V = (double)m.n_vert, T = (double)m.n_tet;
  const bool p2 = m.disp_order == 2;
  const double N = p2 ? 2.0 * V + T : V, n = 3.0 * N;
  const double nnzb = (p2 ? 28.0 : 15.0) * N;
  double bytes = nnzb * (72.0 + 8.0 + 4.0) + nnzb * 0.6 * 4.0 * 8.0;
  if (o.precision == 1 || o.mass_passes) bytes += nnzb * (36.0 + 4.0);
  const double nd = p2 ? 10.0 : 4.0;
  bytes = std::max(bytes, T * nd * nd * 9.0 * 8.0 * 1.5);
  const int bs = o.block > 0 ? o.block : 16;
  for (int i = 0; i < S; ++i) {
    const double K = std::max({6.0 * nev[i], nev[i] + 16.0 * bs, 320.0});
    bytes += 2.0 * K * n * 8.0 + 8.0 * n * bs * 8.0 + 6.0 * n * 3.0 * nev[i] * 8.0;
    if (o.mass_passes) bytes += 4.0 * n * bs * 4.0;  // FP32 work vectors of the mixed mass solve
  }
  return bytes;
}

}  // namespace nm

namespace {

void run_job(nm_server* sv, Job* j) {
  nm_server_result* r = j->res;
  r->t_start = sv->now();
  std::vector<nm_eig_result*> outs(j->a.size(), nullptr);
  hipStream_t st = nullptr;
  nm_pencil* P = nullptr;
  try {
    NM_HIP(hipSetDevice(sv->device));
    NM_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    NM_REQUIRE(nm_assemble(&j->mesh, &j->mat, j->omega, st, &P) == NM_OK, NM_EINVAL,
               std::string("assembly failed: ") + nm_last_error());
    nm_eig_opts o = j->opts;
    o.stream = st;
    const int S = (int)j->a.size();
    std::vector<int> nv(j->nev.begin(), j->nev.end());
    try {
      nm::filtered_eig_slices(P, S, j->a.data(), j->b.data(), nv.data(), j->tol, o, outs.data());
      r->status = NM_OK;
    } catch (const nm::Error& e) {
      if (e.code != NM_PARTIAL) throw;
      r->status = NM_PARTIAL;
    }
    if (j->rotate) {
      // projection over the union of the windows' pairs (one basis)
      int tot = 0;
      for (auto* q : outs) tot += q ? q->count : 0;
      if (tot > 0) {
        nm_eig_result u;
        std::memset(&u, 0, sizeof(u));
        u.count = tot;
        u.n = outs[0]->n;
        std::vector<double> lam(tot), res(tot);
        nm::DBuf<double> X((size_t)u.n * tot);
        int o2 = 0;
        for (auto* q : outs) {
          if (!q || !q->count) continue;
          std::copy(q->lambda, q->lambda + q->count, lam.begin() + o2);
          std::copy(q->resid, q->resid + q->count, res.begin() + o2);
          NM_HIP(hipMemcpy2DAsync(X.p + o2, 8 * (size_t)tot, q->X, 8 * (size_t)q->count, 8 * (size_t)q->count, u.n,
                                  hipMemcpyDeviceToDevice, st));
          o2 += q->count;
        }
        u.lambda = lam.data();
        u.resid = res.data();
        u.X = X.p;
        double lo = 1e300, hi = -1e300;
        for (size_t i = 0; i < j->a.size(); ++i) {
          lo = std::min(lo, j->a[i]);
          hi = std::max(hi, j->b[i]);
        }
        nm::project_rotation(P, &u, lo, hi, st, &r->rotation);
      }
    }
  } catch (const std::exception& e) {
    const nm::Error* ne = dynamic_cast<const nm::Error*>(&e);
    r->status = ne ? ne->code : NM_EDEVICE;
    std::snprintf(r->error, sizeof(r->error), "%s", e.what());
    for (auto*& q : outs) {
      nm_result_free(q);
      q = nullptr;
    }
  }
  if (P) nm_pencil_free(P);
  if (st) (void)hipStreamDestroy(st);
  r->nslices = (int32_t)outs.size();
  r->slices = (nm_eig_result**)std::calloc(std::max<size_t>(outs.size(), 1), sizeof(nm_eig_result*));
  for (size_t i = 0; i < outs.size(); ++i) r->slices[i] = outs[i];
  r->t_end = sv->now();
  std::lock_guard<std::mutex> lk(sv->mx);
  sv->in_use -= j->est;
  --sv->active;
  j->done = true;
  sv->cv.notify_all();
}

void scheduler(nm_server* sv) {
  std::unique_lock<std::mutex> lk(sv->mx);
  for (;;) {
    sv->cv.wait(lk, [&] {
      if (sv->stopping && sv->queue.empty()) return true;
      if (sv->queue.empty() || sv->active >= sv->max_active) return false;
      Job* h = sv->queue.front();
      return sv->active == 0 || sv->in_use + h->est <= sv->budget;
    });
    if (sv->stopping && sv->queue.empty()) return;
    Job* j = sv->queue.front();
    sv->queue.pop_front();
    sv->in_use += j->est;
    ++sv->active;
    j->th = std::thread(run_job, sv, j);
  }
}

}  // namespace

extern "C" {

nm_status nm_server_create(double hbm_budget_bytes, int32_t max_active, nm_server** out) {
  NM_TRY({
    NM_REQUIRE(out && hbm_budget_bytes > 0 && max_active >= 1, NM_EINVAL, "invalid server arguments");
    nm_server* sv = new nm_server();
    sv->budget = hbm_budget_bytes;
    sv->max_active = max_active;
    NM_HIP(hipGetDevice(&sv->device));
    sv->sched = std::thread(scheduler, sv);
    *out = sv;
  })
}

nm_status nm_server_submit(nm_server* sv, const nm_request* q, int64_t* ticket) {
  NM_TRY({
    NM_REQUIRE(sv && q && ticket && q->nslices >= 1 && q->nslices <= 64 && q->a && q->b && q->nev && q->tol > 0,
               NM_EINVAL, "invalid request");
    const nm_mesh& m = q->mesh;
    const nm_material& mt = q->material;
    NM_REQUIRE(m.xyz && m.tet && m.region && mt.rho && mt.lam && mt.mu && m.n_vert > 0 && m.n_tet > 0, NM_EINVAL,
               "request without mesh or material");
    {
      std::lock_guard<std::mutex> lk(sv->mx);
      NM_REQUIRE(!sv->stopping, NM_EINVAL, "server is shutting down");
    }
    std::unique_ptr<Job> jp(new Job());
    Job* j = jp.get();
    const int64_t V = m.n_vert, T = m.n_tet;
    j->xyz.assign(m.xyz, m.xyz + 3 * V);
    j->tet.assign(m.tet, m.tet + 4 * T);
    j->region.assign(m.region, m.region + T);
    j->rho.assign(mt.rho, mt.rho + T);
    j->lam.assign(mt.lam, mt.lam + T);
    j->mu.assign(mt.mu, mt.mu + T);
    j->mesh = m;
    j->mesh.xyz = j->xyz.data();
    j->mesh.tet = j->tet.data();
    j->mesh.region = j->region.data();
    j->mat = mt;
    j->mat.rho = j->rho.data();
    j->mat.lam = j->lam.data();
    j->mat.mu = j->mu.data();
    if (mt.gprime && mt.grad_gprime) {
      const size_t k = (size_t)T * mt.gprime_np;
      j->gp.assign(mt.gprime, mt.gprime + 3 * k);
      j->dgp.assign(mt.grad_gprime, mt.grad_gprime + 9 * k);
      j->mat.gprime = j->gp.data();
      j->mat.grad_gprime = j->dgp.data();
    } else {
      j->mat.gprime = nullptr;
      j->mat.grad_gprime = nullptr;
    }
    for (int i = 0; i < 3; ++i) j->omega[i] = q->omega[i];
    j->a.assign(q->a, q->a + q->nslices);
    j->b.assign(q->b, q->b + q->nslices);
    j->nev.assign(q->nev, q->nev + q->nslices);
    j->tol = q->tol;
    j->opts = q->opts;
    j->rotate = q->rotate;
    j->est = nm::request_bytes(j->mesh, q->nslices, q->nev, q->opts);
    std::lock_guard<std::mutex> lk(sv->mx);
    NM_REQUIRE(!sv->stopping, NM_EINVAL, "server is shutting down");
    j->res = (nm_server_result*)std::calloc(1, sizeof(nm_server_result));
    NM_REQUIRE(j->res, NM_ENOMEM, "host allocation failed");
    j->res->est_bytes = j->est;
    jp.release();  // owned by the server from here on
    j->id = sv->next_id++;
    j->res->t_submit = sv->now();
    sv->jobs[j->id] = j;
    sv->queue.push_back(j);
    *ticket = j->id;
    sv->cv.notify_all();
  })
}

nm_status nm_server_wait(nm_server* sv, int64_t ticket, nm_server_result** out) {
  NM_TRY({
    NM_REQUIRE(sv && out, NM_EINVAL, "invalid arguments");
    Job* j = nullptr;
    {
      std::unique_lock<std::mutex> lk(sv->mx);
      auto it = sv->jobs.find(ticket);
      NM_REQUIRE(it != sv->jobs.end(), NM_EINVAL, "unknown ticket (or already waited for)");
      j = it->second;
      // claim the ticket before waiting: a second waiter on it gets NM_EINVAL
      sv->jobs.erase(it);
      sv->cv.wait(lk, [&] { return j->done; });
    }
    if (j->th.joinable()) j->th.join();
    *out = j->res;
    delete j;
  })
}

void nm_server_result_free(nm_server_result* r) {
  if (!r) return;
  for (int i = 0; i < r->nslices; ++i) nm_result_free(r->slices[i]);
  std::free(r->slices);
  nm_rot_result_free(r->rotation);
  std::free(r);
}

nm_status nm_server_destroy(nm_server* sv) {
  NM_TRY({
    if (!sv) return NM_OK;
    {
      std::lock_guard<std::mutex> lk(sv->mx);
      sv->stopping = true;
      sv->cv.notify_all();
    }
    if (sv->sched.joinable()) sv->sched.join();
    std::vector<Job*> left;
    {
      std::unique_lock<std::mutex> lk(sv->mx);
      sv->cv.wait(lk, [&] { return sv->active == 0; });
      for (auto& kv : sv->jobs) left.push_back(kv.second);
      sv->jobs.clear();
    }
    for (Job* j : left) {
      if (j->th.joinable()) j->th.join();
      nm_server_result_free(j->res);
      delete j;
    }
    delete sv;
  })
}

}  // extern "C"
