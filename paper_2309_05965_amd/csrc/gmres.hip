// Step S6 -- GMRES driver kernels (Alg. 1 Steps 2 and 4).
//
// Unrestarted GMRES with modified Gram-Schmidt and Givens rotations; the
// stopping test |g_{k}| <= tol |b| is taken on the host from one scalar
// read back per iteration.  The Krylov basis V[j][n] and the Hessenberg
// columns live in device memory; every reduction is a fixed-order tree in
// one work group, so results are bitwise reproducible run to run.
#include <math.h>

#include "kfbi_internal.h"

namespace {

constexpr int GB = 1024;

// block-wide sum, fixed order; every thread gets the total
__device__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = GB / 2; off > 0; off >>= 1) {
    if (threadIdx.x < (unsigned)off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  double t = sh[0];
  __syncthreads();
  return t;
}

// r0 = b - A x0 (or b); beta = |r0|; V0 = r0 / beta; g0 = beta; scal[1] = |b|
__global__ void __launch_bounds__(GB) k_start(int64_t n, const double* b, const double* Ax0, double* V,
                                             double* gv, double* scal) {
  __shared__ double sh[GB];
  double sb = 0.0, sr = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += GB) {
    double r = Ax0 ? b[i] - Ax0[i] : b[i];
    V[i] = r;
    sb += b[i] * b[i];
    sr += r * r;
  }
  double nb = sqrt(block_sum(sb, sh));
  double beta = sqrt(block_sum(sr, sh));
  double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  for (int64_t i = threadIdx.x; i < n; i += GB) V[i] = V[i] * inv;
  if (threadIdx.x == 0) {
    gv[0] = beta;
    scal[0] = beta;
    scal[1] = nb;
    scal[2] = 0.0;
  }
}

// Arnoldi step j: w = V[j+1] (holds A V[j]) orthogonalised against V[0..j]
// by MGS, normalised, then the Givens rotations are applied to column j.
__global__ void __launch_bounds__(GB) k_arnoldi(int64_t n, int j, int ldh, double* V, double* Hm, double* cs,
                                               double* sn, double* gv, double* scal) {
  __shared__ double sh[GB];
  double* w = V + (int64_t)(j + 1) * n;
  double* hcol = Hm + (int64_t)j * ldh;
  for (int i = 0; i <= j; ++i) {
    const double* vi = V + (int64_t)i * n;
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < n; t += GB) s += w[t] * vi[t];
    double hij = block_sum(s, sh);
    for (int64_t t = threadIdx.x; t < n; t += GB) w[t] = w[t] - hij * vi[t];
    if (threadIdx.x == 0) hcol[i] = hij;
    __syncthreads();
  }
  double s = 0.0;
  for (int64_t t = threadIdx.x; t < n; t += GB) s += w[t] * w[t];
  double hn = sqrt(block_sum(s, sh));
  bool breakdown = !(hn > 0.0);
  if (!breakdown) {
    double inv = 1.0 / hn;
    for (int64_t t = threadIdx.x; t < n; t += GB) w[t] = w[t] * inv;
  }
  if (threadIdx.x == 0) {
    hcol[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
      double t = cs[i] * hcol[i] + sn[i] * hcol[i + 1];
      hcol[i + 1] = -sn[i] * hcol[i] + cs[i] * hcol[i + 1];
      hcol[i] = t;
    }
    double den = hypot(hcol[j], hcol[j + 1]);
    cs[j] = hcol[j] / den;
    sn[j] = hcol[j + 1] / den;
    hcol[j] = den;
    hcol[j + 1] = 0.0;
    gv[j + 1] = -sn[j] * gv[j];
    gv[j] = cs[j] * gv[j];
    scal[0] = fabs(gv[j + 1]);
    scal[2] = breakdown ? 1.0 : 0.0;
  }
}

// y = H^{-1} g (upper triangular, k x k), then x = x0 + V^T y
__global__ void k_trisolve(int k, int ldh, const double* Hm, const double* gv, double* y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    double s = gv[i];
    for (int m = i + 1; m < k; ++m) s -= Hm[(int64_t)m * ldh + i] * y[m];
    y[i] = s / Hm[(int64_t)i * ldh + i];
  }
}

__global__ void k_combine(int64_t n, int k, const double* V, const double* y, double* x, int use_x0) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = use_x0 ? x[i] : 0.0;
  for (int m = 0; m < k; ++m) s += V[(int64_t)m * n + i] * y[m];
  x[i] = s;
}

__global__ void __launch_bounds__(GB) k_resid(int64_t n, const double* b, const double* Ax, double* out) {
  __shared__ double sh[GB];
  double sr = 0.0, sb = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += GB) {
    double r = b[i] - Ax[i];
    sr += r * r;
    sb += b[i] * b[i];
  }
  double a = block_sum(sr, sh);
  double c = block_sum(sb, sh);
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = c;
  }
}

}  // namespace

void gm_residual_start(kfbi_plan* pl, const double* b, const double* Ax0, int use_x0) {
  hipLaunchKernelGGL(k_start, dim3(1), dim3(GB), 0, pl->stream, pl->n_dof, b, use_x0 ? Ax0 : nullptr, pl->V,
                     pl->gv, pl->scal);
}

void gm_arnoldi(kfbi_plan* pl, int j) {
  hipLaunchKernelGGL(k_arnoldi, dim3(1), dim3(GB), 0, pl->stream, pl->n_dof, j, pl->gm_cap + 1, pl->V, pl->Hm,
                     pl->cs, pl->sn, pl->gv, pl->scal);
}

void gm_update(kfbi_plan* pl, int k, double* x, int use_x0) {
  if (k > 0) hipLaunchKernelGGL(k_trisolve, dim3(1), dim3(64), 0, pl->stream, k, pl->gm_cap + 1, pl->Hm, pl->gv,
                                pl->scal + 8);
  unsigned nbk = (unsigned)((pl->n_dof + KFBI_BLOCK - 1) / KFBI_BLOCK);
  hipLaunchKernelGGL(k_combine, dim3(nbk), dim3(KFBI_BLOCK), 0, pl->stream, pl->n_dof, k, pl->V, pl->scal + 8, x,
                     use_x0);
}

void gm_true_residual(kfbi_plan* pl, const double* b, const double* Ax, double* out2) {
  hipLaunchKernelGGL(k_resid, dim3(1), dim3(GB), 0, pl->stream, pl->n_dof, b, Ax, out2);
}
