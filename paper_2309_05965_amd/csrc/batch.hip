// Step S9 -- many independent interface problems of uneven grid sizes.
//
// A batch owns a pool of workers.  Each worker is a host thread with its
// own HIP stream (default priority) and one plan per grid shape it has
// met; the workers pull problems from a shared counter in order of
// decreasing node count (largest first, so the tail of the batch is made
// of small problems), re-run S0 + S1 on the plan for the problem's
// geometry, generate the manufactured data on the device and run the
// whole solve (Alg. 1) on their stream.  Host-side waits of one worker
// (compaction counts, GMRES convergence checks) overlap with the other
// workers' kernels, so several problems share the GPU at every moment.
//
// Manufactured solutions (fhat_s = Lap u_s - kappa u_s):
//   KFBI_MANU_STAR2D   u_in = cos 2x e^y, u_out = x^2 - y^3         (2D)
//   KFBI_MANU_TORUS3D  u_in = sin x sin y sin z, u_out = e^(x+y+z)/10 (3D)
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

void kfbi_pde_lattice(int d, int p, int (*off)[3], int* n);

namespace {

// value, gradient and Laplacian of region s's solution (s > 0 inside)
__device__ void manu_eval(int kind, int s, const double* x, double& v, double* g, double& lap) {
  if (kind == KFBI_MANU_STAR2D) {
    if (s > 0) {
      const double c = cos(2.0 * x[0]), sn = sin(2.0 * x[0]), e = exp(x[1]);
      v = c * e;
      g[0] = -2.0 * sn * e;
      g[1] = c * e;
      lap = -3.0 * c * e;
    } else {
      v = x[0] * x[0] - x[1] * x[1] * x[1];
      g[0] = 2.0 * x[0];
      g[1] = -3.0 * x[1] * x[1];
      lap = 2.0 - 6.0 * x[1];
    }
    g[2] = 0.0;
  } else {
    if (s > 0) {
      const double sx = sin(x[0]), sy = sin(x[1]), sz = sin(x[2]);
      v = sx * sy * sz;
      g[0] = cos(x[0]) * sy * sz;
      g[1] = sx * cos(x[1]) * sz;
      g[2] = sx * sy * cos(x[2]);
      lap = -3.0 * v;
    } else {
      const double e = exp(x[0] + x[1] + x[2]) / 10.0;
      v = e;
      g[0] = g[1] = g[2] = e;
      lap = 3.0 * e;
    }
  }
}

struct ManuArgs {
  int kind, d, K, nP;
  double kappa, beta_in, beta_out, lo, h;
  int n1;
  int64_t n_surf, n_dof, n_nodes;
  const double *spos, *snrm;
  const int *meta, *d2s;
  int off[KFBI_MAXP][3];
  double *g1, *g2, *ft, *fhat, *gB;
};

__global__ void k_manu_surface(ManuArgs a) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_surf) return;
  const int k = a.meta[i * 5 + 3];
  double x[3] = {0.0, 0.0, 0.0};
  for (int ax = 0; ax < a.d; ++ax) x[ax] = a.spos[i * a.d + ax];
  double vk, gk[3], lk, v0, g0[3], l0;
  manu_eval(a.kind, k, x, vk, gk, lk);
  manu_eval(a.kind, 0, x, v0, g0, l0);
  double dk = 0.0, d0 = 0.0;
  for (int ax = 0; ax < a.d; ++ax) {
    dk += gk[ax] * a.snrm[i * a.d + ax];
    d0 += g0[ax] * a.snrm[i * a.d + ax];
  }
  a.g1[i] = vk - v0;
  a.g2[i] = a.beta_in * dk - a.beta_out * d0;
}

__global__ void k_manu_grid(ManuArgs a) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.n_nodes) return;
  double x[3] = {0.0, 0.0, 0.0};
  int64_t r = q;
  for (int ax = 0; ax < a.d; ++ax) {
    x[ax] = a.lo + (double)(r % a.n1) * a.h;
    r /= a.n1;
  }
  double v, g[3], lap;
  for (int s = 0; s <= a.K; ++s) {
    manu_eval(a.kind, s, x, v, g, lap);
    a.fhat[(int64_t)s * a.n_nodes + q] = lap - a.kappa * v;
    if (s == 0) a.gB[q] = v;
  }
}

__global__ void k_manu_pde(ManuArgs a) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.n_dof * a.nP) return;
  const int64_t c = t / a.nP;
  const int j = (int)(t % a.nP);
  const int s = a.d2s[c];
  const int k = a.meta[(int64_t)s * 5 + 3];
  double x[3] = {0.0, 0.0, 0.0};
  for (int ax = 0; ax < a.d; ++ax) x[ax] = a.spos[(int64_t)s * a.d + ax] + (double)a.off[j][ax] * a.h;
  double vk, gk[3], lk, v0, g0[3], l0;
  manu_eval(a.kind, k, x, vk, gk, lk);
  manu_eval(a.kind, 0, x, v0, g0, l0);
  a.ft[t] = (lk - a.kappa * vk) - (l0 - a.kappa * v0);
}

inline unsigned nbk(int64_t n) { return (unsigned)((n + 255) / 256); }

kfbi_status manufactured(kfbi_plan* pl, int kind, double* g1, double* g2, double* ft, double* fhat, double* gB) {
  if ((kind == KFBI_MANU_STAR2D && pl->g.d != 2) || (kind == KFBI_MANU_TORUS3D && pl->g.d != 3) ||
      (kind != KFBI_MANU_STAR2D && kind != KFBI_MANU_TORUS3D)) {
    kfbi_set_error("manufactured solution %d does not fit a %dD plan", kind, pl->g.d);
    return KFBI_E_INVALID;
  }
  ManuArgs a;
  a.kind = kind;
  a.d = pl->g.d;
  a.K = pl->g.K;
  a.kappa = pl->g.kappa;
  a.beta_in = pl->g.beta_in;
  a.beta_out = pl->g.beta_out;
  a.lo = pl->g.lo;
  a.h = pl->g.h;
  a.n1 = pl->g.n1;
  a.n_surf = pl->n_surf;
  a.n_dof = pl->n_dof;
  a.n_nodes = pl->g.n_nodes;
  a.spos = pl->s_pos;
  a.snrm = pl->s_nrm;
  a.meta = pl->s_meta;
  a.d2s = pl->d2s;
  kfbi_pde_lattice(a.d, pl->g.p, a.off, &a.nP);
  a.g1 = g1;
  a.g2 = g2;
  a.ft = ft;
  a.fhat = fhat;
  a.gB = gB;
  hipStream_t st = pl->stream;
  if (a.n_surf > 0) hipLaunchKernelGGL(k_manu_surface, dim3(nbk(a.n_surf)), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_manu_grid, dim3(nbk(a.n_nodes)), dim3(256), 0, st, a);
  if (a.n_dof > 0) hipLaunchKernelGGL(k_manu_pde, dim3(nbk(a.n_dof * a.nP)), dim3(256), 0, st, a);
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

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
  double *g1 = nullptr, *g2 = nullptr, *ft = nullptr, *fhat = nullptr, *gB = nullptr, *psi = nullptr, *u = nullptr;
  int64_t c_g1 = 0, c_g2 = 0, c_ft = 0, c_fhat = 0, c_gB = 0, c_psi = 0, c_u = 0;
};

std::vector<double> shape_key(const kfbi_problem& p) {
  return {(double)p.dim, (double)p.order, (double)p.N, (double)p.n_iface, p.lo, p.hi};
}

}  // namespace

struct kfbi_batch {
  std::vector<kfbi_problem> probs;
  std::vector<int> manu;
  std::vector<int64_t> u_off;
  std::vector<Worker> workers;
  int device = 0;
};

extern "C" kfbi_status kfbi_batch_create(const kfbi_problem* probs, const int* manu, int n, int n_workers,
                                         kfbi_batch** out) {
  if (!probs || !manu || !out || n < 1 || n_workers < 1 || n_workers > 16) {
    kfbi_set_error("batch needs problems, solution kinds, n >= 1 and 1..16 workers");
    return KFBI_E_INVALID;
  }
  kfbi_batch* b = new (std::nothrow) kfbi_batch();
  if (!b) return KFBI_E_OOM;
  b->probs.assign(probs, probs + n);
  b->manu.assign(manu, manu + n);
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

extern "C" kfbi_status kfbi_batch_solve(kfbi_batch* b, const kfbi_opts* opts, double* u_all, kfbi_info* infos,
                                        double* seconds) {
  if (!b || !opts || !infos) {
    kfbi_set_error("batch solve needs a batch, options and an info array");
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
      if (st == KFBI_OK) {
        std::shared_lock<std::shared_mutex> lock(kfbi_capture_mutex);
        const int64_t nP = pl->nP;
        if ((st = grow(&w.g1, &w.c_g1, pl->n_surf)) == KFBI_OK && (st = grow(&w.g2, &w.c_g2, pl->n_surf)) == KFBI_OK &&
            (st = grow(&w.ft, &w.c_ft, pl->n_dof * nP)) == KFBI_OK &&
            (st = grow(&w.fhat, &w.c_fhat, (int64_t)(prob.n_iface + 1) * nn)) == KFBI_OK &&
            (st = grow(&w.gB, &w.c_gB, nn)) == KFBI_OK && (st = grow(&w.psi, &w.c_psi, pl->n_dof)) == KFBI_OK &&
            (u_all || (st = grow(&w.u, &w.c_u, nn)) == KFBI_OK))
          st = manufactured(pl, b->manu[p], w.g1, w.g2, w.ft, w.fhat, w.gB);
      }
      if (st == KFBI_OK) {
        kfbi_data data{w.g1, w.g2, w.ft, w.fhat, w.gB};
        kfbi_opts o = *opts;
        o.use_x0 = 0;
        st = kfbi_solve(pl, &data, &o, w.psi, u_all ? u_all + b->u_off[p] : w.u, &info);
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
    for (double* p : {w.g1, w.g2, w.ft, w.fhat, w.gB, w.psi, w.u})
      if (p) (void)hipFree(p);
    if (w.stream) (void)hipStreamDestroy(w.stream);
  }
  delete b;
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_plan_manufactured_data(kfbi_plan* pl, int kind, double* g1, double* g2, double* ftilde,
                                                   double* fhat, double* gB) {
  if (!pl || !pl->ready || !g1 || !g2 || !ftilde || !fhat || !gB) {
    kfbi_set_error("manufactured data needs a ready plan and five outputs");
    return KFBI_E_INVALID;
  }
  return manufactured(pl, kind, g1, g2, ftilde, fhat, gB);
}
