// Step S9 -- many independent interface problems of uneven grid sizes.
//
// A batch owns a pool of workers.  Each worker is a host thread with its
// own HIP stream (default priority); the workers pull problems from a
// shared counter in order of decreasing node count (largest first, so the
// tail of the batch is made of small problems).  Host-side waits of one
// worker (compaction counts, GMRES convergence checks) overlap with the
// other workers' kernels, so several problems share the GPU at every
// moment.  Set-up then solve: kfbi_batch_setup builds a plan per problem
// (on the worker's stream), the caller fills the data at the plans' query
// points, and kfbi_batch_solve runs every problem on the worker that set
// it up.  Streaming: each worker keeps one plan per grid shape, re-runs
// S0 + S1 on it for every problem and takes the data from the caller's
// callback.
#include <math.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "kfbi_internal.h"

namespace {

template <typename T>
kfbi_status grow(T** p, int64_t* cap, int64_t n) {
  if (n <= *cap && *p) return KFBI_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  int64_t c = n + n / 4 + 256;
  if (hipMalloc((void**)p, sizeof(T) * (size_t)c) != hipSuccess) {
    (void)hipGetLastError();
    kfbi_set_error("device allocation of %lld bytes failed", (long long)(sizeof(T) * c));
    return KFBI_E_OOM;
  }
  *cap = c;
  return KFBI_OK;
}

struct Worker {
  hipStream_t stream = nullptr;
  std::map<std::vector<double>, kfbi_plan*> plans;
  double *psi = nullptr, *u = nullptr;    // density and solution when the caller keeps neither
  int64_t c_psi = 0, c_u = 0;
};

std::vector<double> shape_key(const kfbi_problem& p) {
  return {(double)p.dim, (double)p.order, (double)p.N, (double)p.n_iface, p.lo, p.hi};
}

}  // namespace

struct kfbi_batch {
  std::vector<kfbi_problem> probs;
  std::vector<int64_t> u_off;
  std::vector<Worker> workers;
  int device = 0;
  // set up, then solve: one plan per problem, the worker that built it,
  // the set-up's status
  std::vector<kfbi_plan*> pplan;
  std::vector<int> owner;
  std::vector<kfbi_status> pstat;
  bool setup_done = false;
};

namespace {
// largest problems first
std::vector<int> work_order(const kfbi_batch* b) {
  const int n = (int)b->probs.size();
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return b->u_off[x + 1] - b->u_off[x] > b->u_off[y + 1] - b->u_off[y]; });
  return order;
}

// run fn(worker index, worker) on every worker's thread (the caller's
// thread is worker 0)
template <class F>
void on_workers(kfbi_batch* b, F fn) {
  std::vector<std::thread> th;
  for (size_t i = 1; i < b->workers.size(); ++i) th.emplace_back([&, i] {
    (void)hipSetDevice(b->device);
    fn((int)i, b->workers[i]);
  });
  (void)hipSetDevice(b->device);
  fn(0, b->workers[0]);
  for (auto& t : th) t.join();
}

struct FirstError {
  std::mutex mu;
  std::string msg;
  kfbi_status st = KFBI_OK;
  void note(int p, kfbi_status s) {
    std::lock_guard<std::mutex> g(mu);
    if (st == KFBI_OK) {
      st = s;
      msg = "problem " + std::to_string(p) + ": " + kfbi_last_error();
    }
  }
  kfbi_status done() {
    if (st != KFBI_OK) kfbi_set_error("%s", msg.c_str());
    return st;
  }
};
}  // namespace

extern "C" kfbi_status kfbi_batch_create(const kfbi_problem* probs, int n, int n_workers, kfbi_batch** out) {
  if (!probs || !out || n < 1 || n_workers < 1 || n_workers > 16) {
    kfbi_set_error("batch needs problems, n >= 1 and 1..16 workers");
    return KFBI_E_INVALID;
  }
  for (int i = 0; i < n; ++i)
    if (probs[i].bie == KFBI_BIE_TWO_DENSITY) {
      kfbi_set_error("problem %d: batches take single-density problems", i);
      return KFBI_E_INVALID;
    }
  kfbi_batch* b = new (std::nothrow) kfbi_batch();
  if (!b) return KFBI_E_OOM;
  b->probs.assign(probs, probs + n);
  int64_t off = 0;
  for (int i = 0; i < n; ++i) {
    b->u_off.push_back(off);
    const int64_t n1 = probs[i].N + 1;
    off += probs[i].dim == 3 ? n1 * n1 * n1 : n1 * n1;
  }
  b->u_off.push_back(off);
  HIPCHK(hipGetDevice(&b->device));
  b->workers.resize(n_workers);
  for (auto& w : b->workers)
    if (hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      kfbi_batch_destroy(b);
      kfbi_set_error("stream creation failed");
      return KFBI_E_DEVICE;
    }
  *out = b;
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_batch_sizes(const kfbi_batch* b, int64_t* n_problems, int64_t* total_nodes) {
  if (!b) {
    kfbi_set_error("batch is NULL");
    return KFBI_E_INVALID;
  }
  if (n_problems) *n_problems = (int64_t)b->probs.size();
  if (total_nodes) *total_nodes = b->u_off.back();
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_batch_setup(kfbi_batch* b, kfbi_info* infos, double* seconds) {
  if (!b) {
    kfbi_set_error("batch is NULL");
    return KFBI_E_INVALID;
  }
  const int n = (int)b->probs.size();
  for (kfbi_plan* pl : b->pplan)
    if (pl) kfbi_plan_destroy(pl);
  b->pplan.assign(n, nullptr);
  b->owner.assign(n, 0);
  b->pstat.assign(n, KFBI_E_INVALID);
  const std::vector<int> order = work_order(b);
  std::atomic<int> next(0);
  FirstError fe;
  on_workers(b, [&](int wi, Worker& w) {
    for (;;) {
      const int k = next.fetch_add(1);
      if (k >= n) break;
      const int p = order[k];
      auto t0 = std::chrono::steady_clock::now();
      kfbi_plan* pl = nullptr;
      kfbi_status st = kfbi_plan_create(&b->probs[p], (void*)w.stream, &pl);
      if (st == KFBI_OK && hipStreamSynchronize(w.stream) != hipSuccess) st = KFBI_E_DEVICE;
      if (st != KFBI_OK) {
        fe.note(p, st);
        if (pl) kfbi_plan_destroy(pl);
        pl = nullptr;
      }
      b->pplan[p] = pl;
      b->owner[p] = wi;
      b->pstat[p] = st;
      if (infos) infos[p] = kfbi_info{0, st, 0.0, 0.0};
      if (seconds) seconds[p] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
  });
  b->setup_done = true;
  return fe.done();
}

extern "C" kfbi_status kfbi_batch_plan(kfbi_batch* b, int i, kfbi_plan** out) {
  if (!b || !out || i < 0 || i >= (int)b->probs.size() || !b->setup_done) {
    kfbi_set_error("batch plan needs a set-up batch, a problem index and an output");
    return KFBI_E_INVALID;
  }
  *out = b->pplan[i];
  if (!*out) kfbi_set_error("problem %d did not set up", i);
  return b->pstat[i];
}

// Problems of one dimension solved by one worker go in groups of up to
// GROUP_MAX (largest first, grid sizes mixed) in lockstep (kfbi_solve_group:
// one launch per box-solve pass for the group's problems up to N = 256 and
// one per larger size) when their box solver is the FFT; others one by
// one.
constexpr int GROUP_MAX = 32;

extern "C" kfbi_status kfbi_batch_solve(kfbi_batch* b, const kfbi_opts* opts, const kfbi_data* data, double* const* psi,
                                        double* u_all, kfbi_info* infos, double* seconds) {
  if (!b || !opts || !data || !infos || !b->setup_done) {
    kfbi_set_error("batch solve needs a set-up batch, options, the data and an info array");
    return KFBI_E_INVALID;
  }
  if (opts->start == KFBI_START_LEARNED || (opts->start == KFBI_START_GIVEN && !psi)) {
    kfbi_set_error("batch solve: a learned start is per problem (kfbi_solve); a given start needs psi");
    return KFBI_E_INVALID;
  }
  const std::vector<int> order = work_order(b);
  const bool fft = opts->solver == KFBI_SOLVER_FFT ||
                   (opts->solver == KFBI_SOLVER_PLAN);   // refined per plan below
  FirstError fe;
  on_workers(b, [&](int wi, Worker& w) {
    // this worker's problems that set up, grouped by dimension (largest first)
    std::map<std::vector<double>, std::vector<int>> groups;
    std::vector<std::vector<double>> shapes;
    for (int p : order) {
      if (b->owner[p] != wi) continue;
      if (b->pstat[p] != KFBI_OK) {
        infos[p] = kfbi_info{0, b->pstat[p], 0.0, 0.0};
        if (seconds) seconds[p] = 0.0;
        continue;
      }
      const std::vector<double> key{(double)b->probs[p].dim};
      if (!groups.count(key)) shapes.push_back(key);
      groups[key].push_back(p);
    }
    for (const auto& key : shapes) {
      const std::vector<int>& ps = groups[key];
      for (size_t c0 = 0; c0 < ps.size(); c0 += GROUP_MAX) {
        const int G = (int)std::min(ps.size() - c0, (size_t)GROUP_MAX);
        auto t0 = std::chrono::steady_clock::now();
        std::vector<kfbi_plan*> pls(G);
        std::vector<kfbi_data> dat(G);
        std::vector<double*> pv(G), uv(G);
        kfbi_status st = KFBI_OK;
        int64_t npsi = 0, nu = 0;
        for (int i = 0; i < G; ++i) {
          const int p = ps[c0 + i];
          pls[i] = b->pplan[p];
          dat[i] = data[p];
          if (!(psi && psi[p])) npsi += pls[i]->n_dof;
          if (!u_all) nu += b->u_off[p + 1] - b->u_off[p];
        }
        {
          std::shared_lock<std::shared_mutex> lock(kfbi_capture_mutex);
          if (npsi > 0) st = grow(&w.psi, &w.c_psi, npsi);
          if (st == KFBI_OK && nu > 0) st = grow(&w.u, &w.c_u, nu);
        }
        int64_t op = 0, ou = 0;
        for (int i = 0; i < G && st == KFBI_OK; ++i) {
          const int p = ps[c0 + i];
          if (psi && psi[p]) {
            pv[i] = psi[p];
          } else {
            pv[i] = w.psi + op;
            op += pls[i]->n_dof;
          }
          if (u_all) {
            uv[i] = u_all + b->u_off[p];
          } else {
            uv[i] = w.u + ou;
            ou += b->u_off[p + 1] - b->u_off[p];
          }
        }
        bool grouped = st == KFBI_OK && fft && G > 1;
        for (int i = 0; i < G && grouped; ++i)
          grouped = (opts->solver == KFBI_SOLVER_FFT) || pls[i]->box_solver == KFBI_BOX_FFT;
        std::vector<kfbi_info> inf(G, kfbi_info{0, st, 0.0, 0.0});
        if (st == KFBI_OK && grouped) {
          st = kfbi_solve_group(pls.data(), G, dat.data(), pv.data(), uv.data(), opts, w.stream, inf.data());
          if (st != KFBI_OK)
            for (int i = 0; i < G; ++i)
              if (inf[i].status == KFBI_OK) inf[i].status = st;
        } else if (st == KFBI_OK) {
          for (int i = 0; i < G; ++i) {
            const kfbi_status si = kfbi_solve(pls[i], &dat[i], opts, pv[i], uv[i], &inf[i]);
            if (hipStreamSynchronize(pls[i]->stream) != hipSuccess && si == KFBI_OK)
              inf[i].status = KFBI_E_DEVICE;
            else
              inf[i].status = si;
          }
        }
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (int i = 0; i < G; ++i) {
          const int p = ps[c0 + i];
          infos[p] = inf[i];
          if (seconds) seconds[p] = secs / G;
          if (inf[i].status != KFBI_OK) fe.note(p, (kfbi_status)inf[i].status);
        }
      }
    }
  });
  return fe.done();
}

extern "C" kfbi_status kfbi_batch_solve_stream(kfbi_batch* b, const kfbi_opts* opts, kfbi_batch_data_fn data_fn,
                                               void* ctx, double* u_all, kfbi_info* infos, double* seconds) {
  if (!b || !opts || !data_fn || !infos) {
    kfbi_set_error("batch solve needs a batch, options, a data callback and an info array");
    return KFBI_E_INVALID;
  }
  if (opts->start == KFBI_START_LEARNED) {
    kfbi_set_error("a learned start is per problem: solve such problems with kfbi_solve");
    return KFBI_E_INVALID;
  }
  const int n = (int)b->probs.size();
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return b->u_off[x + 1] - b->u_off[x] > b->u_off[y + 1] - b->u_off[y]; });
  std::atomic<int> next(0);
  std::mutex mu;
  std::string first_err;
  kfbi_status first_st = KFBI_OK;
  auto run = [&](Worker& w) {
    (void)hipSetDevice(b->device);
    for (;;) {
      const int k = next.fetch_add(1);
      if (k >= n) break;
      const int p = order[k];
      const kfbi_problem& prob = b->probs[p];
      auto t0 = std::chrono::steady_clock::now();
      kfbi_info info{0, KFBI_OK, 0.0, 0.0};
      kfbi_status st = KFBI_OK;
      kfbi_plan*& pl = w.plans[shape_key(prob)];
      if (!pl)
        st = kfbi_plan_create(&prob, (void*)w.stream, &pl);
      else
        st = kfbi_plan_setup(pl, &prob);
      const int64_t nn = b->u_off[p + 1] - b->u_off[p];
      kfbi_data data{nullptr, nullptr, nullptr, nullptr, nullptr};
      double* psi = nullptr;
      if (st == KFBI_OK) st = data_fn(ctx, p, pl, (void*)w.stream, &data, &psi);
      if (st == KFBI_OK && !psi) {
        if (opts->start == KFBI_START_GIVEN) {
          kfbi_set_error("KFBI_START_GIVEN needs the initial density from the data callback");
          st = KFBI_E_INVALID;
        } else {
          std::shared_lock<std::shared_mutex> lock(kfbi_capture_mutex);
          st = grow(&w.psi, &w.c_psi, pl->n_dof);
          psi = w.psi;
        }
      }
      if (st == KFBI_OK && !u_all) {
        std::shared_lock<std::shared_mutex> lock(kfbi_capture_mutex);
        st = grow(&w.u, &w.c_u, nn);
      }
      if (st == KFBI_OK) {
        st = kfbi_solve(pl, &data, opts, psi, u_all ? u_all + b->u_off[p] : w.u, &info);
        if (hipStreamSynchronize(w.stream) != hipSuccess && st == KFBI_OK) st = KFBI_E_DEVICE;
      }
      info.status = st;
      infos[p] = info;
      if (seconds) seconds[p] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (st != KFBI_OK) {
        std::lock_guard<std::mutex> g(mu);
        if (first_st == KFBI_OK) {
          first_st = st;
          first_err = "problem " + std::to_string(p) + ": " + kfbi_last_error();
        }
      }
    }
  };
  std::vector<std::thread> th;
  for (size_t i = 1; i < b->workers.size(); ++i) th.emplace_back(run, std::ref(b->workers[i]));
  run(b->workers[0]);
  for (auto& t : th) t.join();
  if (first_st != KFBI_OK) kfbi_set_error("%s", first_err.c_str());
  return first_st;
}

extern "C" kfbi_status kfbi_batch_destroy(kfbi_batch* b) {
  if (!b) return KFBI_OK;
  for (auto& w : b->workers) {
    for (auto& kv : w.plans)
      if (kv.second) kfbi_plan_destroy(kv.second);
    for (double* p : {w.psi, w.u})
      if (p) (void)hipFree(p);
  }
  for (kfbi_plan* pl : b->pplan)
    if (pl) kfbi_plan_destroy(pl);
  for (auto& w : b->workers) {
    if (w.stream) (void)hipStreamDestroy(w.stream);
  }
  delete b;
  return KFBI_OK;
}
