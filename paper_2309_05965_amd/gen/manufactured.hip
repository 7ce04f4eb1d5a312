// Manufactured-solution test data through the public C ABI (see kfbi_gen.h).
#include <hip/hip_runtime.h>
#include <math.h>

#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "kfbi_gen.h"

namespace {

// value, gradient and Laplacian of region s's solution (s > 0 inside)
__device__ void manu_eval(int kind, int s, const double* x, double& v, double* g, double& lap) {
  if (kind == KFBI_GEN_STAR2D) {
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

struct Args {
  int kind, d, K, nP, n1;
  double kappa, beta_in, beta_out, lo, h;
  int64_t n_surf, n_dof, n_nodes;
  const double *spos, *snrm, *pde;
  const int *meta, *d2s;
  double *g1, *g2, *ft, *fhat, *gB;
};

__global__ void k_surface(Args a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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

__global__ void k_grid(Args a) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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

__global__ void k_pde(Args a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.n_dof * a.nP) return;
  const int64_t c = t / a.nP;
  const int k = a.meta[(int64_t)a.d2s[c] * 5 + 3];
  double x[3] = {0.0, 0.0, 0.0};
  for (int ax = 0; ax < a.d; ++ax) x[ax] = a.pde[t * a.d + ax];
  double vk, gk[3], lk, v0, g0[3], l0;
  manu_eval(a.kind, k, x, vk, gk, lk);
  manu_eval(a.kind, 0, x, v0, g0, l0);
  a.ft[t] = (lk - a.kappa * vk) - (l0 - a.kappa * v0);
}

inline unsigned nbk(int64_t n) { return (unsigned)((n + 255) / 256); }

// a thread's device workspace, grown on demand
struct Work {
  std::vector<std::pair<void*, int64_t>> buf;   // pointer, bytes
  void* get(int i, int64_t bytes) {
    if ((int)buf.size() <= i) buf.resize(i + 1, {nullptr, 0});
    if (buf[i].second < bytes || !buf[i].first) {
      if (buf[i].first) (void)hipFree(buf[i].first);
      buf[i] = {nullptr, 0};
      const int64_t c = bytes + bytes / 4 + 256;
      if (hipMalloc(&buf[i].first, (size_t)c) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
      buf[i].second = c;
    }
    return buf[i].first;
  }
};

std::mutex g_mu;
std::map<std::thread::id, Work*> g_work;

Work& my_work() {
  std::lock_guard<std::mutex> g(g_mu);
  Work*& w = g_work[std::this_thread::get_id()];
  if (!w) w = new Work();
  return *w;
}

enum { B_POS, B_NRM, B_META, B_D2S, B_PDE, B_G1, B_G2, B_FT, B_FHAT, B_GB };

kfbi_status plan_data(kfbi_plan* plan, const kfbi_problem* prob, int kind, hipStream_t st, Work& w, double* g1,
                      double* g2, double* ft, double* fhat, double* gB) {
  if ((kind == KFBI_GEN_STAR2D && prob->dim != 2) || (kind == KFBI_GEN_TORUS3D && prob->dim != 3) ||
      (kind != KFBI_GEN_STAR2D && kind != KFBI_GEN_TORUS3D))
    return KFBI_E_INVALID;
  kfbi_sizes sz;
  kfbi_status s = kfbi_plan_sizes(plan, &sz);
  if (s != KFBI_OK) return s;
  const int d = prob->dim;
  Args a;
  a.kind = kind;
  a.d = d;
  a.K = prob->n_iface;
  a.nP = sz.n_pde;
  a.n1 = prob->N + 1;
  a.kappa = prob->kappa;
  a.beta_in = prob->beta_in;
  a.beta_out = prob->beta_out;
  a.lo = prob->lo;
  a.h = sz.h;
  a.n_surf = sz.n_surf;
  a.n_dof = sz.n_dof;
  a.n_nodes = sz.n_nodes;
  const int64_t bpos = 8 * sz.n_surf * d, bmeta = 4 * 5 * sz.n_surf, bd2s = 4 * sz.n_dof,
                bpde = 8 * sz.n_dof * sz.n_pde * d;
  double* pos = (double*)w.get(B_POS, bpos);
  double* nrm = (double*)w.get(B_NRM, bpos);
  int* meta = (int*)w.get(B_META, bmeta);
  int* d2s = (int*)w.get(B_D2S, bd2s);
  double* pde = (double*)w.get(B_PDE, bpde);
  if (!pos || !nrm || !meta || !d2s || !pde) return KFBI_E_OOM;
  // the exports are ordered on the plan's stream, which is `st` here
  if ((s = kfbi_plan_export(plan, KFBI_EXPORT_SURF_POS, pos, bpos)) != KFBI_OK ||
      (s = kfbi_plan_export(plan, KFBI_EXPORT_SURF_NRM, nrm, bpos)) != KFBI_OK ||
      (s = kfbi_plan_export(plan, KFBI_EXPORT_SURF_META, meta, bmeta)) != KFBI_OK ||
      (s = kfbi_plan_export(plan, KFBI_EXPORT_DOF_SURF, d2s, bd2s)) != KFBI_OK ||
      (s = kfbi_plan_export(plan, KFBI_EXPORT_PDE_PTS, pde, bpde)) != KFBI_OK)
    return s;
  a.spos = pos;
  a.snrm = nrm;
  a.meta = meta;
  a.d2s = d2s;
  a.pde = pde;
  a.g1 = g1;
  a.g2 = g2;
  a.ft = ft;
  a.fhat = fhat;
  a.gB = gB;
  if (a.n_surf > 0) hipLaunchKernelGGL(k_surface, dim3(nbk(a.n_surf)), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_grid, dim3(nbk(a.n_nodes)), dim3(256), 0, st, a);
  if (a.n_dof > 0) hipLaunchKernelGGL(k_pde, dim3(nbk(a.n_dof * a.nP)), dim3(256), 0, st, a);
  return hipGetLastError() == hipSuccess ? KFBI_OK : KFBI_E_DEVICE;
}

}  // namespace

struct kfbi_gen {
  std::vector<kfbi_problem> probs;
  std::vector<int> kinds;
  double* psi_all;
  int64_t psi_stride;
};

extern "C" kfbi_status kfbi_gen_plan_data(kfbi_plan* plan, const kfbi_problem* prob, int kind, void* stream,
                                          double* g1, double* g2, double* ftilde, double* fhat, double* gB) {
  if (!plan || !prob || !g1 || !g2 || !ftilde || !fhat || !gB) return KFBI_E_INVALID;
  return plan_data(plan, prob, kind, (hipStream_t)stream, my_work(), g1, g2, ftilde, fhat, gB);
}

extern "C" kfbi_status kfbi_gen_create(const kfbi_problem* probs, const int* kinds, int n, double* psi_all,
                                       int64_t psi_stride, kfbi_gen** out) {
  if (!probs || !kinds || n < 1 || !out || (psi_all && psi_stride < 1)) return KFBI_E_INVALID;
  kfbi_gen* g = new (std::nothrow) kfbi_gen();
  if (!g) return KFBI_E_OOM;
  g->probs.assign(probs, probs + n);
  g->kinds.assign(kinds, kinds + n);
  g->psi_all = psi_all;
  g->psi_stride = psi_stride;
  *out = g;
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_gen_batch_data(void* ctx, int problem, kfbi_plan* plan, void* stream, kfbi_data* data,
                                           double** psi_out) {
  kfbi_gen* g = (kfbi_gen*)ctx;
  if (!g || problem < 0 || problem >= (int)g->probs.size() || !plan || !data || !psi_out) return KFBI_E_INVALID;
  const kfbi_problem& prob = g->probs[problem];
  kfbi_sizes sz;
  kfbi_status s = kfbi_plan_sizes(plan, &sz);
  if (s != KFBI_OK) return s;
  Work& w = my_work();
  double* g1 = (double*)w.get(B_G1, 8 * sz.n_surf);
  double* g2 = (double*)w.get(B_G2, 8 * sz.n_surf);
  double* ft = (double*)w.get(B_FT, 8 * sz.n_dof * sz.n_pde);
  double* fhat = (double*)w.get(B_FHAT, 8 * (int64_t)(prob.n_iface + 1) * sz.n_nodes);
  double* gB = (double*)w.get(B_GB, 8 * sz.n_nodes);
  if (!g1 || !g2 || !ft || !fhat || !gB) return KFBI_E_OOM;
  if ((s = plan_data(plan, &prob, g->kinds[problem], (hipStream_t)stream, w, g1, g2, ft, fhat, gB)) != KFBI_OK)
    return s;
  *data = kfbi_data{g1, g2, ft, fhat, gB};
  *psi_out = nullptr;
  if (g->psi_all) {
    if (sz.n_dof > g->psi_stride) return KFBI_E_INVALID;
    *psi_out = g->psi_all + (int64_t)problem * g->psi_stride;
  }
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_gen_destroy(kfbi_gen* g) {
  delete g;
  return KFBI_OK;
}

extern "C" void kfbi_gen_release(void) {
  std::lock_guard<std::mutex> g(g_mu);
  for (auto& kv : g_work) {
    for (auto& b : kv.second->buf)
      if (b.first) (void)hipFree(b.first);
    delete kv.second;
  }
  g_work.clear();
}
