// Step S6 -- GMRES driver kernels (Alg. 1 Steps 2 and 4).
//
// Unrestarted GMRES (CGS2 Arnoldi, Givens rotations).  The iteration index,
// the stopping test |g_k| <= tol |b| and the iteration count live in a
// device control word, so the host can launch a captured iteration
// (matvec + Arnoldi step) repeatedly and read the state back only now and
// then.  The Krylov basis V[j][n] and the Hessenberg columns live in device
// memory; every reduction has a fixed order, so results are bitwise
// reproducible run to run.
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

// r0 = b - A x0 (or b); beta = |r0|; V0 = r0 / beta; g0 = beta; scal[1] = |b|.
// Initialises the control word ctl = [j = 0, done, k = 0, max_iter] and the
// stopping threshold scal[3] = tol.
__global__ void __launch_bounds__(GB) k_start(int64_t n, const double* b, const double* Ax0, double* V,
                                             double* gv, double* scal, int* ctl, double tol, int maxit) {
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
    scal[3] = tol;
    ctl[0] = 0;
    ctl[1] = (nb == 0.0 || beta <= tol * nb) ? 1 : 0;
    ctl[2] = 0;
    ctl[3] = maxit;
  }
}

// Arnoldi step j: w = V[j+1] (holds A V[j]) is orthogonalised against
// V[0..j] by classical Gram-Schmidt applied twice (CGS2: the j+1 dot
// products of a pass are computed concurrently, one wavefront per basis
// vector, with fixed-order wave reductions), then normalised; the Givens
// rotations are applied to column j.
__device__ __forceinline__ double wave_reduce(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ void __launch_bounds__(GB) k_arnoldi(int64_t n, int* ctl, int ldh, double* V, double* Hm, double* cs,
                                               double* sn, double* gv, double* scal) {
  __shared__ double hp[KFBI_GMRES_MAX + 1];
  __shared__ double hs[KFBI_GMRES_MAX + 1];
  __shared__ double red[GB / 64];
  if (ctl[1]) return;
  const int j = ctl[0];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* w = V + (int64_t)(j + 1) * n;
  double* hcol = Hm + (int64_t)j * ldh;
  for (int pass = 0; pass < 2; ++pass) {
    // one wavefront per basis vector: h_i = <w, V_i>; four independent
    // partial sums per lane keep several loads in flight
    for (int i = wave; i <= j; i += GB / 64) {
      const double* vi = V + (int64_t)i * n;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int64_t t = lane;
      for (; t + 192 < n; t += 256) {
        s0 += w[t] * vi[t];
        s1 += w[t + 64] * vi[t + 64];
        s2 += w[t + 128] * vi[t + 128];
        s3 += w[t + 192] * vi[t + 192];
      }
      for (; t < n; t += 64) s0 += w[t] * vi[t];
      double sacc = wave_reduce((s0 + s1) + (s2 + s3));
      if (lane == 0) hp[i] = sacc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= j; i += GB) hs[i] = pass == 0 ? hp[i] : hs[i] + hp[i];
    for (int64_t t = threadIdx.x; t < n; t += GB) {
      double v = w[t];
#pragma unroll 8
      for (int i = 0; i <= j; ++i) v -= hp[i] * V[(int64_t)i * n + t];
      w[t] = v;
    }
    __syncthreads();
  }
  double sq = 0.0;
  for (int64_t t = threadIdx.x; t < n; t += GB) sq += w[t] * w[t];
  sq = wave_reduce(sq);
  if (lane == 0) red[wave] = sq;
  __syncthreads();
  double tot = 0.0;
  for (int wv = 0; wv < GB / 64; ++wv) tot += red[wv];
  double hn = sqrt(tot);
  bool breakdown = !(hn > 0.0);
  if (!breakdown) {
    double inv = 1.0 / hn;
    for (int64_t t = threadIdx.x; t < n; t += GB) w[t] = w[t] * inv;
  }
  // Givens rotations of column j, in LDS (the previous rotations are read in
  // parallel first; the recurrence itself is sequential)
  __shared__ double lcs[KFBI_GMRES_MAX], lsn[KFBI_GMRES_MAX];
  for (int i = threadIdx.x; i < j; i += GB) {
    lcs[i] = cs[i];
    lsn[i] = sn[i];
  }
  if (threadIdx.x == 0) hs[j + 1] = hn;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < j; ++i) {
      double t = lcs[i] * hs[i] + lsn[i] * hs[i + 1];
      hs[i + 1] = -lsn[i] * hs[i] + lcs[i] * hs[i + 1];
      hs[i] = t;
    }
    double den = hypot(hs[j], hs[j + 1]);
    double cj = hs[j] / den, sj = hs[j + 1] / den;
    cs[j] = cj;
    sn[j] = sj;
    hs[j] = den;
    hs[j + 1] = 0.0;
    double gj = gv[j];
    gv[j + 1] = -sj * gj;
    gv[j] = cj * gj;
    double res = fabs(-sj * gj);
    scal[0] = res;
    scal[2] = breakdown ? 1.0 : 0.0;
    ctl[2] = j + 1;
    ctl[0] = j + 1;
    ctl[1] = (res <= scal[3] * scal[1] || breakdown || j + 1 >= ctl[3]) ? 1 : 0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j + 1; i += GB) hcol[i] = hs[i];
}

// y = H^{-1} g (upper triangular, k x k), then x = x0 + V^T y.  The
// triangle is staged in LDS (k <= 64) so the sequential back substitution
// reads no global memory.
__global__ void __launch_bounds__(256) k_trisolve(int k, int ldh, const double* Hm, const double* gv, double* y) {
  __shared__ double H[64][65];
  __shared__ double gl[64];
  if (k <= 64) {
    for (int t = threadIdx.x; t < k * k; t += blockDim.x) {
      int m = t / k, i = t % k;      // column m, row i
      H[i][m] = Hm[(int64_t)m * ldh + i];
    }
    for (int t = threadIdx.x; t < k; t += blockDim.x) gl[t] = gv[t];
    __syncthreads();
    __shared__ double yl[64];
    if (threadIdx.x == 0) {
      for (int i = k - 1; i >= 0; --i) {
        double s = gl[i];
        for (int m = i + 1; m < k; ++m) s -= H[i][m] * yl[m];
        yl[i] = s / H[i][i];
      }
      for (int i = 0; i < k; ++i) y[i] = yl[i];
    }
    return;
  }
  if (threadIdx.x != 0) return;
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

void gm_residual_start(kfbi_plan* pl, const double* b, const double* Ax0, int use_x0, double tol, int maxit) {
  hipLaunchKernelGGL(k_start, dim3(1), dim3(GB), 0, pl->stream, pl->n_dof, b, use_x0 ? Ax0 : nullptr, pl->V,
                     pl->gv, pl->scal, pl->ctl, tol, maxit);
}

void gm_arnoldi(kfbi_plan* pl) {
  hipLaunchKernelGGL(k_arnoldi, dim3(1), dim3(GB), 0, pl->stream, pl->n_dof, pl->ctl, pl->gm_cap + 1, pl->V, pl->Hm,
                     pl->cs, pl->sn, pl->gv, pl->scal);
}

void gm_update(kfbi_plan* pl, int k, double* x, int use_x0) {
  if (k > 0) hipLaunchKernelGGL(k_trisolve, dim3(1), dim3(256), 0, pl->stream, k, pl->gm_cap + 1, pl->Hm, pl->gv,
                                pl->scal + 8);
  unsigned nbk = (unsigned)((pl->n_dof + KFBI_BLOCK - 1) / KFBI_BLOCK);
  hipLaunchKernelGGL(k_combine, dim3(nbk), dim3(KFBI_BLOCK), 0, pl->stream, pl->n_dof, k, pl->V, pl->scal + 8, x,
                     use_x0);
}

void gm_true_residual(kfbi_plan* pl, const double* b, const double* Ax, double* out2) {
  hipLaunchKernelGGL(k_resid, dim3(1), dim3(GB), 0, pl->stream, pl->n_dof, b, Ax, out2);
}
