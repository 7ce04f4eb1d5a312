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

// dimension and degree of a coefficient count (6, 10, 15, 35)
constexpr int dim_of(int nc) { return nc == 10 || nc == 35 ? 3 : 2; }
constexpr int deg_of(int nc) { return nc == 15 || nc == 35 ? 4 : 2; }

// monomial exponents in graded order, the same order as kfbi_exponents
template <int D, int P>
struct Exponents {
  int e[KFBI_MAXC][3];
  constexpr Exponents() : e{} {
    int n = 0;
    for (int m = 0; m <= P; ++m) {
      if (D == 2) {
        for (int j = 0; j <= m; ++j) {
          e[n][0] = m - j;
          e[n][1] = j;
          e[n][2] = 0;
          ++n;
        }
      } else {
        for (int x = m; x >= 0; --x)
          for (int y = m - x; y >= 0; --y) {
            e[n][0] = x;
            e[n][1] = y;
            e[n][2] = m - x - y;
            ++n;
          }
      }
    }
  }
};

// row j of M (lane j) in the order [PDE | Dirichlet | Neumann], written to
// row[0..NC) (LDS).  Powers xi^e are formed once per row by repeated
// multiplication (the same products, in the same order, as a per-entry
// power loop), and the exponents are compile-time constants, so every
// column is straight-line code.
template <int NC>
__device__ __forceinline__ void assemble_row(const FactorArgs& a, int64_t c, int j, double* row) {
  constexpr int D = dim_of(NC), P = deg_of(NC);
  constexpr Exponents<D, P> EX{};
  const GridDesc& g = a.g;
  const double h = g.h;
  const int s = a.d2s[c];
  const double* Pc = a.spos + (int64_t)s * D;
  double xi[3] = {0.0, 0.0, 0.0}, nv[3] = {0.0, 0.0, 0.0};
  int kind;   // 0 PDE, 1 Dirichlet, 2 Neumann
  if (j < a.T.nP) {
    kind = 0;
    for (int ax = 0; ax < D; ++ax) xi[ax] = (double)a.T.offP[j][ax];
  } else if (j < a.T.nP + a.T.nD) {
    kind = 1;
    int q = a.stD[c * a.T.nD + (j - a.T.nP)];
    for (int ax = 0; ax < D; ++ax) xi[ax] = (a.spos[(int64_t)q * D + ax] - Pc[ax]) / h;
  } else {
    kind = 2;
    int q = a.stN[c * a.T.nN + (j - a.T.nP - a.T.nD)];
    for (int ax = 0; ax < D; ++ax) {
      xi[ax] = (a.spos[(int64_t)q * D + ax] - Pc[ax]) / h;
      nv[ax] = a.snrm[(int64_t)q * D + ax];
    }
  }
  double pw[D][P + 1];
#pragma unroll
  for (int ax = 0; ax < D; ++ax) {
    pw[ax][0] = 1.0;
#pragma unroll
    for (int e = 1; e <= P; ++e) pw[ax][e] = pw[ax][e - 1] * xi[ax];
  }
  const double kh2 = g.kappa * h * h;
#pragma unroll
  for (int al = 0; al < NC; ++al) {
    double v;
    if (kind == 1) {
      v = 1.0;
#pragma unroll
      for (int ax = 0; ax < D; ++ax) v *= pw[ax][EX.e[al][ax]];
    } else if (kind == 2) {
      v = 0.0;
#pragma unroll
      for (int ax = 0; ax < D; ++ax) {
        if (EX.e[al][ax] == 0) continue;
        double t = (double)EX.e[al][ax];
#pragma unroll
        for (int b = 0; b < D; ++b) t *= pw[b][b == ax ? EX.e[al][b] - 1 : EX.e[al][b]];
        v += nv[ax] * t;
      }
    } else {
      double lap = 0.0, val = 1.0;
#pragma unroll
      for (int ax = 0; ax < D; ++ax) val *= pw[ax][EX.e[al][ax]];
#pragma unroll
      for (int ax = 0; ax < D; ++ax) {
        if (EX.e[al][ax] < 2) continue;
        double t = (double)(EX.e[al][ax] * (EX.e[al][ax] - 1));
#pragma unroll
        for (int b = 0; b < D; ++b) t *= pw[b][b == ax ? EX.e[al][b] - 2 : EX.e[al][b]];
        lap += t;
      }
      v = lap - kh2 * val;
    }
    row[al] = v;
  }
}

// value of x in lane l (l uniform across the wavefront)
__device__ __forceinline__ double lane_value(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// One wavefront per centre, lane j holds row j of M in registers and the
// inverse is formed in place (Gauss-Jordan).  Partial pivoting: at step k
// the pivot is the unused row with the largest |entry| in column k (lowest
// lane on ties: a max reduction, then the first lane of the ballot of lanes
// holding it); rows are not swapped.  The pivot lane scales its row
// (column k becomes 1/pivot) and writes it to LDS, and after a barrier the
// other lanes read it (broadcast reads) and eliminate.  With p_k the pivot lane of step k, lane p_a ends up holding
// row a of the inverse with its column j at position p_j.
template <int NC>
__global__ void __launch_bounds__(64) k_factor(FactorArgs a) {
  // a geometry status flag (unresolved stencil, extension or owner) means the
  // stencil tables may hold no valid point: nothing to factor, the host
  // reports the flag after this kernel
  if (*a.flags) return;
  const int64_t c = blockIdx.x;
  const int lane = threadIdx.x;
  const bool live = lane < NC;
  __shared__ double Ms[NC][NC + 1];
  __shared__ int pvt[NC];
  if (live) assemble_row<NC>(a, c, lane, Ms[lane]);
  __syncthreads();
  // M^T (for the refinement of U) and the 1-norm of M (max column sum),
  // both read from LDS
  double* mt = a.MT + c * (int64_t)NC * NC;
  for (int idx = lane; idx < NC * NC; idx += 64) mt[idx] = Ms[idx % NC][idx / NC];
  double normM = 0.0;
  if (live)
    for (int j = 0; j < NC; ++j) normM += fabs(Ms[j][lane]);
  normM = wave_max(normM);
  double row[NC];
#pragma unroll
  for (int al = 0; al < NC; ++al) row[al] = live ? Ms[lane][al] : 0.0;
  bool used = !live;
  int myk = -1;
  bool singular = false;
  // the lanes that hold rows: the pivot search reduces over W lanes
  constexpr int W = NC <= 16 ? 16 : (NC <= 32 ? 32 : 64);
  // the scaled pivot row of step k goes through prow[k & 1]: written by the
  // pivot lane, read by every lane after the barrier (the other buffer is
  // the one the next step writes, so no read of step k races with it)
  __shared__ double prow[2][NC];
  // every step unrolled: column k of the row is a fixed register (a zero
  // or non-finite pivot ends the elimination: the later steps do nothing)
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    if (singular) continue;
    const double rk = row[k];
    // pivot: the largest |value| among unused rows, the lowest lane on ties
    const double best = used ? -1.0 : fabs(rk);
    double mx = best;
    for (int off = W / 2; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    mx = lane_value(mx, 0);
    if (!(mx > 0.0) || !isfinite(mx)) {
      singular = true;
      continue;
    }
    const int pl = __ffsll((unsigned long long)__ballot(best == mx)) - 1;
    if (lane == 0) pvt[k] = pl;
    if (lane == pl) {
      const double ri = 1.0 / rk;
#pragma unroll
      for (int m = 0; m < NC; ++m) row[m] = m == k ? ri : row[m] * ri;
#pragma unroll
      for (int m = 0; m < NC; ++m) prow[k & 1][m] = row[m];
      used = true;
      myk = k;
    }
    __syncthreads();
    // the scaled pivot row from LDS (one broadcast read per entry), eight
    // entries at a time
    const double f = (lane != pl && live) ? rk : 0.0;
#pragma unroll
    for (int m0 = 0; m0 < NC; m0 += 8) {
      double pr[8];
#pragma unroll
      for (int m = m0; m < NC && m < m0 + 8; ++m) pr[m - m0] = prow[k & 1][m];
      if (lane != pl && live) {
#pragma unroll
        for (int m = m0; m < NC && m < m0 + 8; ++m) row[m] = m == k ? -(f * pr[m - m0]) : row[m] - f * pr[m - m0];
      }
    }
  }
  if (singular) {
    if (lane == 0) {
      atomicOr(a.flags, FLAG_SINGULAR);
      a.cond[c] = INFINITY;
    }
    return;
  }
  // the in-place result back to LDS: Ms[lane][j] = Minv[myk][p_j]
  __syncthreads();
  if (live) {
#pragma unroll
    for (int j = 0; j < NC; ++j) Ms[lane][j] = row[j];
  }
  __shared__ int rowof[NC];       // lane holding row alpha of the inverse
  if (live) rowof[myk] = lane;
  __syncthreads();
  // 1-norm of the inverse (column sums are invariant under the row and
  // column permutation of the in-place result)
  double normI = 0.0;
  if (live)
    for (int i = 0; i < NC; ++i) normI += fabs(Ms[i][lane]);
  normI = wave_max(normI);
  if (lane == 0) {
    const double cn = normM * normI;
    a.cond[c] = cn;
    if (!(cn <= 1e10)) atomicOr(a.flags, FLAG_SINGULAR);
  }
  // MinvT[c][j][alpha] = Minv[alpha][j]; column j of Minv is column q of
  // the in-place result with p_q = j
  __shared__ int colof[NC];
  if (live) colof[pvt[lane]] = lane;
  __syncthreads();
  double* out = a.MinvT + c * (int64_t)NC * NC;
  for (int idx = lane; idx < NC * NC; idx += 64) {
    const int j = idx / NC, al = idx % NC;
    out[idx] = Ms[rowof[al]][colof[j]];
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
  // the status flags hold the geometry's (cleared at its start, read back
  // here together with the factorisation's): k_factor does nothing if one
  // is set
  FactorArgs a{pl->g, T, pl->n_dof, pl->d2s, pl->s_pos, pl->s_nrm, pl->stD, pl->stN, pl->MinvT, pl->MT,
               pl->cond, pl->d_flags};
  switch (T.n) {
    case 6: hipLaunchKernelGGL(k_factor<6>, dim3((unsigned)pl->n_dof), dim3(64), 0, pl->stream, a); break;
    case 10: hipLaunchKernelGGL(k_factor<10>, dim3((unsigned)pl->n_dof), dim3(64), 0, pl->stream, a); break;
    case 15: hipLaunchKernelGGL(k_factor<15>, dim3((unsigned)pl->n_dof), dim3(64), 0, pl->stream, a); break;
    case 35: hipLaunchKernelGGL(k_factor<35>, dim3((unsigned)pl->n_dof), dim3(64), 0, pl->stream, a); break;
    default:
      kfbi_set_error("no collocation kernel for %d coefficients", T.n);
      return KFBI_E_INVALID;
  }
  HIPCHK(hipGetLastError());
  // flags and the largest condition number (a NaN wins): posted now, read
  // by colloc_finish after the folds have been enqueued
  PostReq& q = pl->colloc_req;
  q = PostReq{};
  q.ni = 1;
  q.isrc[0] = pl->d_flags;
  q.maxsrc = pl->cond;
  q.nmax = pl->n_dof;
  return kfbi_post_launch(pl, q, &pl->colloc_seq);
}

kfbi_status colloc_finish(kfbi_plan* pl) {
  int fl = 0;
  double cm = 0.0;
  KCHK(kfbi_post_collect(pl, pl->colloc_req, pl->colloc_seq, &fl, &cm));
  pl->cond_max = cm;
  if (fl) return kfbi_flags_status(fl);
  return KFBI_OK;
}
