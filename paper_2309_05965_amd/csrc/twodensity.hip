// Two-density interface BIE (eq. bie-ifp-1, Sec. 3.2): the interface problem
// with different reduced reaction coefficients kappa~_1 = kappa_1 / sigma_1
// inside and kappa~_2 = kappa_2 / sigma_2 outside.  Unknowns phi = u_1 and
// psi = sigma_2 d_n u_2 at the DOFs, [phi; psi] of length 2 n_dof.
//
// W_i(a, b, F; gB) is the simple interface problem (Sec. 4) of Lap -
// kappa~_i with [W] = a, [d_n W] = b.  u_1 1_Omega_1 = W_1(u_1, d_n u_1,
// fhat_1 1_Omega_1) and u_2 1_Omega_2 = W_2(-u_2, -d_n u_2, fhat_2 1_Omega_2;
// gB); the averages (in + out)/2 of their traces and of sigma_i times their
// normal derivatives, added in pairs, are eq. bie-ifp-1 with u_2 = phi - g1,
// d_n u_1 = (psi + g2)/sigma_1, d_n u_2 = psi/sigma_2:
//   A [phi; psi] = [phi - avg W_1(phi, psi/s1) + avg W_2(phi, psi/s2);
//                   psi - s1 avg d_n W_1(phi, psi/s1) + s2 avg d_n W_2(phi, psi/s2)]
//   b = [g1/2 + avg R_1 + avg R_2; -g2/2 + s1 avg d_n R_1 + s2 avg d_n R_2],
//   R_1 = W_1(0, g2/s1, fhat_1 1_Omega_1), R_2 = W_2(g1, 0, fhat_2 1_Omega_2; gB).
// Every product is one simple solve per Green's function, i.e. two box
// solves (the superposition remark after Alg. 1).  The plan holds W_1 (its
// own kappa) and keeps a second plan of the same geometry for W_2
// (kappa_out).  In a product both solves run the folded operator, whose
// weight lists cover both densities (phi through the value columns, psi
// through the flux columns); the right-hand side and the final solution use
// the general simple-solve kernels.  The one-sided values come from the
// value weights of the interpolation blocks, the normal derivatives from the
// derivative weights.
//
// GMRES (Alg. 1 Steps 2-4) on the 2 n_dof system: classical Gram-Schmidt
// applied twice, with the dot products reduced on the device in a fixed
// order and the Hessenberg matrix and Givens rotations on the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "kfbi_internal.h"

#pragma clang fp contract(off)

namespace {

constexpr int TD_BLOCK = 256;
constexpr int TD_PARTS = 128;   // fixed number of partial sums per dot product

template <class T>
kfbi_status td_regrow(T** p, int64_t n) {
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  if (n < 1) n = 1;
  if (hipMalloc((void**)p, (size_t)n * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    kfbi_set_error("device allocation of %lld bytes failed", (long long)(n * sizeof(T)));
    return KFBI_E_OOM;
  }
  return KFBI_OK;
}

unsigned nblocks(int64_t n) { return (unsigned)((n + TD_BLOCK - 1) / TD_BLOCK); }

// out = [phi - v1 + v2; psi - s1 d1 + s2 d2] with v_i, d_i the averages of
// the one-sided values and normal derivatives of W_i
__global__ void k_td_combine(int64_t n, const double* x, const double* vi1, const double* vo1, const double* di1,
                             const double* do1, const double* vi2, const double* vo2, const double* di2,
                             const double* do2, double s1, double s2, double* out) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const double v1 = 0.5 * (vi1[c] + vo1[c]), v2 = 0.5 * (vi2[c] + vo2[c]);
  const double d1 = 0.5 * (di1[c] + do1[c]), d2 = 0.5 * (di2[c] + do2[c]);
  out[c] = x[c] - v1 + v2;
  out[n + c] = x[n + c] - s1 * d1 + s2 * d2;
}

// b = [g1/2 + v1 + v2; -g2/2 + s1 d1 + s2 d2] at the DOFs
__global__ void k_td_rhs(int64_t n, const int* d2s, const double* g1, const double* g2, const double* vi1,
                         const double* vo1, const double* di1, const double* do1, const double* vi2,
                         const double* vo2, const double* di2, const double* do2, double s1, double s2,
                         double* out) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const double v1 = 0.5 * (vi1[c] + vo1[c]), v2 = 0.5 * (vi2[c] + vo2[c]);
  const double d1 = 0.5 * (di1[c] + do1[c]), d2 = 0.5 * (di2[c] + do2[c]);
  const int s = d2s[c];
  const double a = g1 ? g1[s] : 0.0, b = g2 ? g2[s] : 0.0;
  out[c] = 0.5 * a + v1 + v2;
  out[n + c] = -0.5 * b + s1 * d1 + s2 * d2;
}

// out = x + alpha y on the surface table (y may be null: out = x)
__global__ void k_td_axpy(int64_t n, const double* x, double alpha, const double* y, double* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = y ? x[i] + alpha * y[i] : x[i];
}

// u = u_1 at the interior nodes, u_2 elsewhere
__global__ void k_td_select(int64_t n, const int8_t* region, const double* u1, const double* u2, double* u) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  u[i] = region[i] != 0 ? u1[i] : u2[i];
}

// partial dot products part[v][blk] = sum over blk's share of V_v . w
// (V_v = V + v * n; fixed split, fixed order)
__global__ void __launch_bounds__(TD_BLOCK) k_td_dots(int64_t n, const double* V, const double* w, double* part) {
  __shared__ double red[TD_BLOCK];
  const int v = blockIdx.y;
  const double* a = V + (int64_t)v * n;
  const int64_t chunk = (n + TD_PARTS - 1) / TD_PARTS;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  int64_t hi = lo + chunk;
  if (hi > n) hi = n;
  double s = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += TD_BLOCK) s += a[i] * w[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = TD_BLOCK / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)v * TD_PARTS + blockIdx.x] = red[0];
}

__global__ void k_td_dots_final(int nv, const double* part, double* out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  double s = 0.0;
  for (int b = 0; b < TD_PARTS; ++b) s += part[(int64_t)v * TD_PARTS + b];
  out[v] = s;
}

// w = w + sign * sum_v h[v] V_v (v in order)
__global__ void k_td_combo(int64_t n, int nv, const double* V, const double* h, double sign, double* w) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int v = 0; v < nv; ++v) s += h[v] * V[(int64_t)v * n + i];
  w[i] = w[i] + sign * s;
}

__global__ void k_td_scale(int64_t n, const double* x, double a, double* y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  y[i] = a * x[i];
}

// one simple solve of the plan P with both kinds of one-sided limits at the
// DOFs: v, (vin, vout) values, (P->dn_in, P->dn_out) normal derivatives
void td_simple(kfbi_plan* P, const double* a, const double* b, double bscale, const double* ftilde, double fscale,
               const double* fhat, int fsel, const double* gB, double* v) {
  op_coefficients(P, a, b, ftilde, bscale, fscale);
  op_correction_values(P);
  op_rhs_base(P, fhat, gB, P->Fs, true, fsel);
  plan_box_solve(P, P->Fs, v);
  op_boundary(P, gB, v);
  op_normal_derivatives(P, v, P->dn_in, P->dn_out, nullptr);
  op_values(P, v, P->tv_in, P->tv_out);
}

kfbi_status td_buffers(kfbi_plan* P) {
  if (P->n_dof > P->td_cap_dof) {
    const int64_t cap = P->cap_dof;
    P->td_cap_dof = 0;
    KCHK(td_regrow(&P->tv_in, cap));
    KCHK(td_regrow(&P->tv_out, cap));
    P->td_cap_dof = cap;
  }
  return KFBI_OK;
}

kfbi_status td_gmres_buffers(kfbi_plan* pl, int m) {
  const int64_t n2 = 2 * pl->cap_dof;
  if (m <= pl->td_m && n2 <= pl->td_n && pl->td_V) return KFBI_OK;
  const int mm = m > pl->td_m ? m : pl->td_m;
  pl->td_m = 0;
  KCHK(td_regrow(&pl->td_V, (int64_t)(mm + 1) * n2));
  KCHK(td_regrow(&pl->td_b, n2));
  KCHK(td_regrow(&pl->td_w, n2));
  KCHK(td_regrow(&pl->td_part, (int64_t)(mm + 1) * TD_PARTS));
  KCHK(td_regrow(&pl->td_h, mm + 1));
  if (pl->h_td) (void)hipHostFree(pl->h_td);
  pl->h_td = nullptr;
  if (hipHostMalloc((void**)&pl->h_td, sizeof(double) * (mm + 1), 0) != hipSuccess) {
    (void)hipGetLastError();
    kfbi_set_error("pinned host allocation failed");
    return KFBI_E_OOM;
  }
  pl->td_m = mm;
  pl->td_n = n2;
  return KFBI_OK;
}

// V_0..V_{nv-1} . w (device, into td_h and the pinned host copy), waits
kfbi_status td_dots(kfbi_plan* pl, int64_t n, const double* V, int nv, const double* w, double* host) {
  hipLaunchKernelGGL(k_td_dots, dim3(TD_PARTS, nv), dim3(TD_BLOCK), 0, pl->stream, n, V, w, pl->td_part);
  hipLaunchKernelGGL(k_td_dots_final, dim3((nv + 63) / 64), dim3(64), 0, pl->stream, nv, pl->td_part, pl->td_h);
  HIPCHK(hipMemcpyAsync(pl->h_td, pl->td_h, sizeof(double) * nv, hipMemcpyDeviceToHost, pl->stream));
  HIPCHK(hipStreamSynchronize(pl->stream));
  for (int v = 0; v < nv; ++v) host[v] = pl->h_td[v];
  return KFBI_OK;
}

kfbi_status td_norm(kfbi_plan* pl, int64_t n, const double* w, double* out) {
  double s = 0.0;
  KCHK(td_dots(pl, n, w, 1, w, &s));
  *out = std::sqrt(s);
  return KFBI_OK;
}

}  // namespace

kfbi_status td_setup(kfbi_plan* pl) {
  kfbi_problem q = pl->prob;
  q.kappa = pl->prob.kappa_out;
  if (!pl->aux) {
    KCHK(plan_create_impl(&q, pl->stream, &pl->aux, true));
  } else {
    pl->aux->stream = pl->stream;
    KCHK(plan_resetup(pl->aux, &q));
  }
  if (pl->aux->n_dof != pl->n_dof || pl->aux->n_surf != pl->n_surf) {
    kfbi_set_error("two-density set-up: the exterior plan's geometry differs");
    return KFBI_E_DEVICE;
  }
  KCHK(td_buffers(pl));
  KCHK(td_buffers(pl->aux));
  return KFBI_OK;
}

void td_free(kfbi_plan* pl) {
  if (pl->aux) plan_release(pl->aux);
  pl->aux = nullptr;
  double** bufs[] = {&pl->IWv, &pl->TIv, &pl->GWv, &pl->HWv, &pl->tv_in, &pl->tv_out, &pl->td_V, &pl->td_b, &pl->td_w, &pl->td_part,
                     &pl->td_h};
  for (double** b : bufs) {
    if (*b) (void)hipFree(*b);
    *b = nullptr;
  }
  if (pl->h_td) (void)hipHostFree(pl->h_td);
  pl->h_td = nullptr;
}

namespace {
kfbi_status td_check(kfbi_plan* pl) {
  if (pl->g.bie != KFBI_BIE_TWO_DENSITY || !pl->aux) {
    kfbi_set_error("not a two-density plan");
    return KFBI_E_INVALID;
  }
  if (pl->box_solver != KFBI_BOX_FFT) {
    kfbi_set_error("the two-density form uses the FFT box solver");
    return KFBI_E_INVALID;
  }
  pl->aux->stream = pl->stream;
  return KFBI_OK;
}

// out = A x (both [2 n_dof], distinct): per Green's function the folded
// operator (the density extension and the local inverses folded at set-up
// into weight lists over [phi; psi]): correction values, the box solve that
// builds the corrected right-hand side in its first pass, and the two
// interpolations
void td_apply(kfbi_plan* pl, const double* x, double* out) {
  kfbi_plan* q = pl->aux;
  const int64_t n = pl->n_dof;
  const double s1 = pl->prob.beta_in, s2 = pl->prob.beta_out;
  for (kfbi_plan* P : {pl, q}) {
    op_matvec_head(P, x);
    dst_solve_corrections(P, x, P->vbuf);
    op_interp_folded(P, P->vbuf, x, P->dn_in, P->dn_out, false);
    op_interp_folded(P, P->vbuf, x, P->tv_in, P->tv_out, true);
  }
  hipLaunchKernelGGL(k_td_combine, dim3(nblocks(n)), dim3(TD_BLOCK), 0, pl->stream, n, x, pl->tv_in, pl->tv_out,
                     pl->dn_in, pl->dn_out, q->tv_in, q->tv_out, q->dn_in, q->dn_out, s1, s2, out);
}

void td_rhs_impl(kfbi_plan* pl, const kfbi_data& d, double* b) {
  kfbi_plan* q = pl->aux;
  const int64_t n = pl->n_dof;
  const double s1 = pl->prob.beta_in, s2 = pl->prob.beta_out;
  const double* ft1 = d.ftilde;
  const double* ft2 = d.ftilde ? d.ftilde + n * pl->nP : nullptr;
  // R_1 = W_1(0, g2/s1, fhat_1 1_Omega_1): its jump in F is fhat_1
  td_simple(pl, nullptr, d.g2, 1.0 / s1, ft1, 1.0, d.fhat, 1, nullptr, pl->vsbuf);
  // R_2 = W_2(g1, 0, fhat_2 1_Omega_2; gB): its jump in F is -fhat_2
  td_simple(q, d.g1, nullptr, 1.0, ft2, -1.0, d.fhat, 2, d.gB, q->vsbuf);
  hipLaunchKernelGGL(k_td_rhs, dim3(nblocks(n)), dim3(TD_BLOCK), 0, pl->stream, n, pl->d2s, d.g1, d.g2, pl->tv_in,
                     pl->tv_out, pl->dn_in, pl->dn_out, q->tv_in, q->tv_out, q->dn_in, q->dn_out, s1, s2, b);
}

// u_1 = W_1(phi, (psi + g2)/s1, fhat_1 1_Omega_1) inside, u_2 = W_2(g1 - phi,
// -psi/s2, fhat_2 1_Omega_2; gB) outside
void td_final(kfbi_plan* pl, const kfbi_data& d, const double* x, double* u) {
  kfbi_plan* q = pl->aux;
  const int64_t n = pl->n_dof, ns = pl->n_surf;
  const double s1 = pl->prob.beta_in, s2 = pl->prob.beta_out;
  const double* ft1 = d.ftilde;
  const double* ft2 = d.ftilde ? d.ftilde + n * pl->nP : nullptr;
  op_extend(pl, x, pl->aS);
  op_extend(pl, x + n, pl->psiS);
  // psiS + g2 and g1 - aS, in the aux plan's surface buffers
  hipLaunchKernelGGL(k_td_axpy, dim3(nblocks(ns)), dim3(TD_BLOCK), 0, pl->stream, ns, pl->psiS, 1.0, d.g2,
                     q->psiS);
  if (d.g1)
    hipLaunchKernelGGL(k_td_axpy, dim3(nblocks(ns)), dim3(TD_BLOCK), 0, pl->stream, ns, d.g1, -1.0, pl->aS, q->aS);
  else
    hipLaunchKernelGGL(k_td_scale, dim3(nblocks(ns)), dim3(TD_BLOCK), 0, pl->stream, ns, pl->aS, -1.0, q->aS);
  td_simple(pl, pl->aS, q->psiS, 1.0 / s1, ft1, 1.0, d.fhat, 1, nullptr, pl->vsbuf);
  td_simple(q, q->aS, pl->psiS, -1.0 / s2, ft2, -1.0, d.fhat, 2, d.gB, q->vsbuf);
  hipLaunchKernelGGL(k_td_select, dim3(nblocks(pl->g.n_nodes)), dim3(TD_BLOCK), 0, pl->stream, pl->g.n_nodes,
                     pl->region, pl->vsbuf, q->vsbuf, u);
}
}  // namespace

kfbi_status td_matvec(kfbi_plan* pl, const double* x, double* out) {
  KCHK(td_check(pl));
  td_apply(pl, x, out);
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

kfbi_status td_rhs(kfbi_plan* pl, const kfbi_data* d, double* b) {
  KCHK(td_check(pl));
  td_rhs_impl(pl, *d, b);
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

kfbi_status td_solve(kfbi_plan* pl, const kfbi_data* d, const kfbi_opts* o, double* x, double* u,
                     kfbi_info* info) {
  KCHK(td_check(pl));
  const int m = o->max_iter;
  const double tol = o->tol > 0.0 ? o->tol : 1e-10;
  if (m < 1 || m > KFBI_GMRES_MAX) {
    kfbi_set_error("max_iter must be in [1, %d]", KFBI_GMRES_MAX);
    return KFBI_E_INVALID;
  }
  if (o->start != KFBI_START_ZERO && o->start != KFBI_START_GIVEN) {
    kfbi_set_error("the two-density form takes a zero or a given start");
    return KFBI_E_INVALID;
  }
  KCHK(td_gmres_buffers(pl, m));
  const int64_t n2 = 2 * pl->n_dof;
  const unsigned nb2 = nblocks(n2);
  hipStream_t st = pl->stream;
  double* V = pl->td_V;
  double* w = pl->td_w;
  double* b = pl->td_b;
  // Step 1: right-hand side; Step 2: r0 = b - A x0 into V_0
  td_rhs_impl(pl, *d, b);
  const bool given = o->start == KFBI_START_GIVEN;
  if (given) {
    td_apply(pl, x, w);
    hipLaunchKernelGGL(k_td_axpy, dim3(nb2), dim3(TD_BLOCK), 0, st, n2, b, -1.0, w, V);
  } else {
    HIPCHK(hipMemcpyAsync(V, b, sizeof(double) * n2, hipMemcpyDeviceToDevice, st));
  }
  double nb = 0.0, beta = 0.0;
  KCHK(td_norm(pl, n2, b, &nb));
  KCHK(td_norm(pl, n2, V, &beta));
  if (!std::isfinite(nb) || !std::isfinite(beta)) {
    kfbi_set_error("non-finite right-hand side or initial residual");
    if (info) *info = kfbi_info{0, KFBI_E_NONFINITE, NAN, NAN};
    return KFBI_E_NONFINITE;
  }
  std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m, 0.0), sn(m, 0.0), g(m + 1, 0.0), h1(m + 1), h2(m + 1);
  g[0] = beta;
  int k = 0;
  bool conv = nb == 0.0 || beta <= tol * nb;
  if (!conv && beta > 0.0)
    hipLaunchKernelGGL(k_td_scale, dim3(nb2), dim3(TD_BLOCK), 0, st, n2, V, 1.0 / beta, V);
  for (int j = 0; j < m && !conv; ++j) {
    double* vj = V + (int64_t)j * n2;
    double* wj = V + (int64_t)(j + 1) * n2;
    td_apply(pl, vj, wj);
    // classical Gram-Schmidt, twice
    KCHK(td_dots(pl, n2, V, j + 1, wj, h1.data()));
    HIPCHK(hipMemcpyAsync(pl->td_h, h1.data(), sizeof(double) * (j + 1), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_td_combo, dim3(nb2), dim3(TD_BLOCK), 0, st, n2, j + 1, V, pl->td_h, -1.0, wj);
    KCHK(td_dots(pl, n2, V, j + 1, wj, h2.data()));
    HIPCHK(hipMemcpyAsync(pl->td_h, h2.data(), sizeof(double) * (j + 1), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_td_combo, dim3(nb2), dim3(TD_BLOCK), 0, st, n2, j + 1, V, pl->td_h, -1.0, wj);
    double hn = 0.0;
    KCHK(td_norm(pl, n2, wj, &hn));
    if (!std::isfinite(hn)) {
      kfbi_set_error("non-finite Krylov vector");
      if (info) *info = kfbi_info{j, KFBI_E_NONFINITE, NAN, NAN};
      return KFBI_E_NONFINITE;
    }
    double* col = &H[(size_t)j * (m + 1)];
    for (int i = 0; i <= j; ++i) col[i] = h1[i] + h2[i];
    col[j + 1] = hn;
    const bool breakdown = !(hn > 0.0);
    if (!breakdown) hipLaunchKernelGGL(k_td_scale, dim3(nb2), dim3(TD_BLOCK), 0, st, n2, wj, 1.0 / hn, wj);
    for (int i = 0; i < j; ++i) {
      const double t = cs[i] * col[i] + sn[i] * col[i + 1];
      col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
      col[i] = t;
    }
    const double den = std::hypot(col[j], col[j + 1]);
    cs[j] = col[j] / den;
    sn[j] = col[j + 1] / den;
    col[j] = den;
    col[j + 1] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    k = j + 1;
    conv = std::fabs(g[j + 1]) <= tol * nb;
    if (breakdown) break;
  }
  // x = x0 + V y
  std::vector<double> y(k > 0 ? k : 1, 0.0);
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int l = i + 1; l < k; ++l) s -= H[(size_t)l * (m + 1) + i] * y[l];
    y[i] = s / H[(size_t)i * (m + 1) + i];
  }
  if (!given) HIPCHK(hipMemsetAsync(x, 0, sizeof(double) * n2, st));
  if (k > 0) {
    HIPCHK(hipMemcpyAsync(pl->td_h, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_td_combo, dim3(nb2), dim3(TD_BLOCK), 0, st, n2, k, V, pl->td_h, 1.0, x);
  }
  // true residual and the solution
  td_apply(pl, x, w);
  hipLaunchKernelGGL(k_td_axpy, dim3(nb2), dim3(TD_BLOCK), 0, st, n2, b, -1.0, w, w);
  double rn = 0.0;
  KCHK(td_norm(pl, n2, w, &rn));
  if (u) td_final(pl, *d, x, u);
  HIPCHK(hipGetLastError());
  const double est = nb > 0.0 ? std::fabs(g[k]) / nb : 0.0;
  const double tr = nb > 0.0 ? rn / nb : rn;
  kfbi_status s = KFBI_OK;
  if (!std::isfinite(tr)) {
    s = KFBI_E_NONFINITE;
    kfbi_set_error("non-finite residual");
  } else if (!conv) {
    s = KFBI_E_NOT_CONVERGED;
    kfbi_set_error("GMRES did not reach tol %g in %d iterations (estimate %g)", tol, k, est);
  }
  if (info) *info = kfbi_info{k, s, est, tr};
  if (u) HIPCHK(hipStreamSynchronize(st));
  return s;
}
