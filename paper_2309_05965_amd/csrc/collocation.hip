// Step S1 -- batched collocation for the local Cauchy problems.
//
// Paper: Sec. 5.3 (restricted local Cauchy problems, eq. local-cau-prb),
// Sec. 5.3.1 (Taylor monomials in the scaled coordinates xi = (x - p_i)/h,
// eqs. cau-appro / cau-ls), Sec. 5.4 (square system: PDE points on a
// degree p-2 lattice, Dirichlet points of degree p and Neumann points of
// degree p-1 in the reference plane; solved by a standard factorisation).
//
// Every centre owns one wavefront: the n x n system (n <= 35) is built in
// LDS next to an identity block and inverted by Gauss-Jordan elimination
// with partial pivoting (lane i owns row i).  The inverse is stored
// transposed per centre, Minv^T[c][j][alpha], so that the per-matvec
// coefficient kernel reads it with consecutive lanes on consecutive alpha.
// The 1-norm condition number is kept for diagnostics; cond > 1e10 (or a
// zero pivot) flags the plan singular.
#include <math.h>

#include <vector>

#include "kfbi_internal.h"

// every entry of M is formed by plain multiplications and additions in a
// fixed order (no contraction), so the matrices are bitwise reproducible
#pragma clang fp contract(off)

void kfbi_pde_lattice(int d, int p, int (*off)[3], int* n);

namespace {

struct CollocTables {
  int n, nP, nD, nN, d;
  int E[KFBI_MAXC][3];        // monomial exponents, graded order
  int offP[KFBI_MAXP][3];     // PDE lattice
};

__device__ __forceinline__ double ipow(double x, int e) {
  double r = 1.0;
  for (int i = 0; i < e; ++i) r *= x;
  return r;
}

struct FactorArgs {
  GridDesc g;
  CollocTables T;
  int64_t n_dof;
  const int* d2s;
  const double *spos, *snrm;
  const int *stD, *stN;
  double* MinvT;
  double* MT;         // M^T[c][alpha][j] (kept for the refinement of U)
  double* cond;
  int* flags;
};

__global__ void __launch_bounds__(64) k_factor(FactorArgs a) {
  const int n = a.T.n;
  const int d = a.T.d;
  const int64_t c = blockIdx.x;
  const int lane = threadIdx.x;
  __shared__ double A[KFBI_MAXC][2 * KFBI_MAXC + 1];
  __shared__ double colsum[KFBI_MAXC];
  __shared__ int piv;
  const GridDesc& g = a.g;
  const double h = g.h;
  const int s = a.d2s[c];
  const double* P = a.spos + (int64_t)s * d;
  if (lane < n) {
    const int j = lane;
    double xi[3] = {0.0, 0.0, 0.0}, nv[3] = {0.0, 0.0, 0.0};
    int kind;   // 0 PDE, 1 Dirichlet, 2 Neumann
    if (j < a.T.nP) {
      kind = 0;
      for (int ax = 0; ax < d; ++ax) xi[ax] = (double)a.T.offP[j][ax];
    } else if (j < a.T.nP + a.T.nD) {
      kind = 1;
      int q = a.stD[c * a.T.nD + (j - a.T.nP)];
      for (int ax = 0; ax < d; ++ax) xi[ax] = (a.spos[(int64_t)q * d + ax] - P[ax]) / h;
    } else {
      kind = 2;
      int q = a.stN[c * a.T.nN + (j - a.T.nP - a.T.nD)];
      for (int ax = 0; ax < d; ++ax) {
        xi[ax] = (a.spos[(int64_t)q * d + ax] - P[ax]) / h;
        nv[ax] = a.snrm[(int64_t)q * d + ax];
      }
    }
    const double kh2 = g.kappa * h * h;
    for (int al = 0; al < n; ++al) {
      const int* e = a.T.E[al];
      double v;
      if (kind == 1) {
        v = 1.0;
        for (int ax = 0; ax < d; ++ax) v *= ipow(xi[ax], e[ax]);
      } else if (kind == 2) {
        v = 0.0;
        for (int ax = 0; ax < d; ++ax) {
          if (e[ax] == 0) continue;
          double t = (double)e[ax];
          for (int b = 0; b < d; ++b) t *= ipow(xi[b], b == ax ? e[b] - 1 : e[b]);
          v += nv[ax] * t;
        }
      } else {
        double lap = 0.0, val = 1.0;
        for (int ax = 0; ax < d; ++ax) val *= ipow(xi[ax], e[ax]);
        for (int ax = 0; ax < d; ++ax) {
          if (e[ax] < 2) continue;
          double t = (double)(e[ax] * (e[ax] - 1));
          for (int b = 0; b < d; ++b) t *= ipow(xi[b], b == ax ? e[b] - 2 : e[b]);
          lap += t;
        }
        v = lap - kh2 * val;
      }
      A[j][al] = v;
      A[j][n + al] = al == j ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  {
    double* mt = a.MT + c * (int64_t)n * n;
    for (int idx = lane; idx < n * n; idx += 64) {
      int al = idx / n, j = idx % n;
      mt[idx] = A[j][al];
    }
  }
  // 1-norm of M (max column sum)
  if (lane < n) {
    double t = 0.0;
    for (int i = 0; i < n; ++i) t += fabs(A[i][lane]);
    colsum[lane] = t;
  }
  __syncthreads();
  double normM = 0.0;
  for (int i = 0; i < n; ++i) normM = fmax(normM, colsum[i]);
  bool singular = false;
  for (int k = 0; k < n; ++k) {
    if (lane == 0) {
      int p = k;
      double best = fabs(A[k][k]);
      for (int i = k + 1; i < n; ++i)
        if (fabs(A[i][k]) > best) {
          best = fabs(A[i][k]);
          p = i;
        }
      piv = p;
    }
    __syncthreads();
    int p = piv;
    if (p != k)
      for (int m = lane; m < 2 * n; m += 64) {
        double t = A[k][m];
        A[k][m] = A[p][m];
        A[p][m] = t;
      }
    __syncthreads();
    double pv = A[k][k];
    if (pv == 0.0 || !isfinite(pv)) {
      singular = true;
      break;
    }
    __syncthreads();
    for (int m = lane; m < 2 * n; m += 64) A[k][m] = A[k][m] / pv;
    __syncthreads();
    if (lane < n && lane != k) {
      double f = A[lane][k];
      if (f != 0.0)
        for (int m = 0; m < 2 * n; ++m) A[lane][m] -= f * A[k][m];
    }
    __syncthreads();
  }
  if (singular) {
    if (lane == 0) {
      atomicOr(a.flags, FLAG_SINGULAR);
      a.cond[c] = INFINITY;
    }
    return;
  }
  if (lane < n) {
    double t = 0.0;
    for (int i = 0; i < n; ++i) t += fabs(A[i][n + lane]);
    colsum[lane] = t;
  }
  __syncthreads();
  if (lane == 0) {
    double ni = 0.0;
    for (int i = 0; i < n; ++i) ni = fmax(ni, colsum[i]);
    double cn = normM * ni;
    a.cond[c] = cn;
    if (!(cn <= 1e10)) atomicOr(a.flags, FLAG_SINGULAR);
  }
  // Minv[alpha][j] = A[alpha][n + j]  ->  MinvT[c][j][alpha]
  double* out = a.MinvT + c * (int64_t)n * n;
  for (int idx = lane; idx < n * n; idx += 64) {
    int j = idx / n, al = idx % n;
    out[idx] = A[al][n + j];
  }
}

}  // namespace

void kfbi_exponents(int d, int p, int (*E)[3], int* n) {
  *n = 0;
  for (int m = 0; m <= p; ++m) {
    if (d == 2) {
      for (int j = 0; j <= m; ++j) {
        E[*n][0] = m - j;
        E[*n][1] = j;
        E[*n][2] = 0;
        ++*n;
      }
    } else {
      for (int x = m; x >= 0; --x)
        for (int y = m - x; y >= 0; --y) {
          E[*n][0] = x;
          E[*n][1] = y;
          E[*n][2] = m - x - y;
          ++*n;
        }
    }
  }
}

kfbi_status colloc_factor(kfbi_plan* pl) {
  CollocTables T;
  T.d = pl->g.d;
  kfbi_exponents(T.d, pl->g.p, T.E, &T.n);
  kfbi_pde_lattice(T.d, pl->g.p, T.offP, &T.nP);
  T.nD = pl->nD;
  T.nN = pl->nN;
  if (T.n != pl->nC || T.nP + T.nD + T.nN != T.n) {
    kfbi_set_error("collocation sizes inconsistent (%d %d %d %d)", T.n, T.nP, T.nD, T.nN);
    return KFBI_E_INVALID;
  }
  HIPCHK(hipMemsetAsync(pl->d_flags, 0, sizeof(int), pl->stream));
  FactorArgs a{pl->g, T, pl->n_dof, pl->d2s, pl->s_pos, pl->s_nrm, pl->stD, pl->stN, pl->MinvT, pl->MT,
               pl->cond, pl->d_flags};
  hipLaunchKernelGGL(k_factor, dim3((unsigned)pl->n_dof), dim3(64), 0, pl->stream, a);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(pl->h_pinned + 1, pl->d_flags, sizeof(int), hipMemcpyDeviceToHost, pl->stream));
  HIPCHK(hipStreamSynchronize(pl->stream));
  // largest condition number (host reduction of a small array)
  std::vector<double> cond((size_t)pl->n_dof);
  HIPCHK(hipMemcpy(cond.data(), pl->cond, sizeof(double) * pl->n_dof, hipMemcpyDeviceToHost));
  double cm = 0.0;
  for (double v : cond) cm = v > cm || v != v ? v : cm;
  pl->cond_max = cm;
  if (pl->h_pinned[1]) return kfbi_flags_status(pl->h_pinned[1]);
  return KFBI_OK;
}
