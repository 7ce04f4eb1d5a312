// Steps S2, S4, S5 of the BIE operator and the right-hand-side assembly.
//
// Paper:
//  * Sec. 5.3: correction function by the closest-primary-point partition
//    of unity, C_h(x) = C_{h,i*(x)}(x), one polynomial per centre;
//  * Sec. 5.2, eqs. corrected-FDS / crc-formula and the multi-crossing
//    remark: at an irregular node P of region s the right-hand side gets
//    - sum_{Q in S_P, reg Q = t != s} c_PQ (C^(s) - C^(t))(x_Q), C^(0) = 0;
//  * Sec. 5.5: the one-sided normal derivative at a surface point is the
//    derivative of the Lagrange interpolant of grid values made smooth by
//    adding C^(k) - C^(reg q) at nodes q outside interface k's interior;
//  * Sec. 3.2: the flux jump J = beta_in d_n w_in - beta_out d_n w_out
//    gives A psi = J / (beta_in + beta_out) = psi/2 + mu K' psi.
//
// All kernels are gathers (one thread per output), so no atomics and the
// results are bitwise deterministic.
#include <math.h>

#include "kfbi_internal.h"

// discrete decisions (interpolation blocks) must match the rules bit for bit
#pragma clang fp contract(off)

void kfbi_exponents(int d, int p, int (*E)[3], int* n);
void kfbi_pde_lattice(int d, int p, int (*off)[3], int* n);

namespace {

struct Mono {
  int n, d, p;
  int E[KFBI_MAXC][3];
};

struct Stencil {            // A_h and B_h on the 3^d cube, index (o0+1) + 3 (o1+1) + 9 (o2+1)
  double A[27], B[27];
};

inline unsigned nb(int64_t n, int b = KFBI_BLOCK) { return (unsigned)((n + b - 1) / b); }

Mono make_mono(const kfbi_plan* pl) {
  Mono m;
  m.d = pl->g.d;
  m.p = pl->g.p;
  kfbi_exponents(m.d, m.p, m.E, &m.n);
  return m;
}

// compact FD operator A_h = L_h - kappa B_h and B_h (Sec. 5.2, eqs. 9p-cds /
// 27p-cds in tensor form; order 2: Lap_5/7 - kappa I, B = I)
Stencil make_stencil(const GridDesc& g) {
  Stencil S;
  double h2 = g.h * g.h;
  auto D = [&](int o) { return (o == 0 ? -2.0 : 1.0) / h2; };
  auto I = [](int o) { return o == 0 ? 1.0 : 0.0; };
  int zr = g.d == 3 ? 1 : 0;
  for (int i = 0; i < 27; ++i) S.A[i] = S.B[i] = 0.0;
  for (int o2 = -zr; o2 <= zr; ++o2)
    for (int o1 = -1; o1 <= 1; ++o1)
      for (int o0 = -1; o0 <= 1; ++o0) {
        int o[3] = {o0, o1, o2};
        double lap = 0.0, ident = 1.0;
        for (int a = 0; a < g.d; ++a) {
          double t = D(o[a]);
          for (int b = 0; b < g.d; ++b)
            if (b != a) t *= I(o[b]);
          lap += t;
          ident *= I(o[a]);
        }
        double L, B;
        if (g.order == 2) {
          L = lap;
          B = ident;
        } else {
          L = lap;
          for (int a = 0; a < g.d; ++a)
            for (int b = a + 1; b < g.d; ++b) {
              double t = D(o[a]) * D(o[b]);
              for (int c = 0; c < g.d; ++c)
                if (c != a && c != b) t *= I(o[c]);
              L += h2 / 6.0 * t;
            }
          if (g.d == 3) L += h2 * h2 / 48.0 * D(o[0]) * D(o[1]) * D(o[2]);
          B = ident + h2 / 12.0 * lap;
        }
        int idx = (o0 + 1) + 3 * (o1 + 1) + 9 * (o2 + 1);
        S.A[idx] = L - g.kappa * B;
        S.B[idx] = B;
      }
  return S;
}

__device__ __forceinline__ void unravel(const GridDesc& g, int64_t idx, int c[3]) {
  c[0] = (int)(idx % g.n1);
  int64_t r = idx / g.n1;
  c[1] = (int)(r % g.n1);
  c[2] = g.d == 3 ? (int)(r / g.n1) : 0;
}

__device__ __forceinline__ int64_t ravel(const GridDesc& g, int c0, int c1, int c2) {
  return (int64_t)c0 + (int64_t)g.n1 * ((int64_t)c1 + (g.d == 3 ? (int64_t)g.n1 * c2 : 0));
}

__device__ __forceinline__ double Cval(const double* Cg, int64_t n, int k, int64_t q) {
  return k == 0 ? 0.0 : Cg[(int64_t)(k - 1) * n + q];
}

// monomials xi^alpha of total degree <= P in graded order (fully unrolled,
// so every index is a compile-time constant)
template <int D, int P>
__device__ __forceinline__ void monomials(const double xi[3], double* phi) {
  double px[P + 1], py[P + 1], pz[P + 1];
  px[0] = py[0] = pz[0] = 1.0;
#pragma unroll
  for (int e = 1; e <= P; ++e) {
    px[e] = px[e - 1] * xi[0];
    py[e] = py[e - 1] * xi[1];
    pz[e] = D == 3 ? pz[e - 1] * xi[2] : 0.0;
  }
  int n = 0;
#pragma unroll
  for (int m = 0; m <= P; ++m) {
    if (D == 2) {
#pragma unroll
      for (int j = 0; j <= m; ++j) phi[n++] = px[m - j] * py[j];
    } else {
#pragma unroll
      for (int x = m; x >= 0; --x)
#pragma unroll
        for (int y = m - x; y >= 0; --y) phi[n++] = px[x] * py[y] * pz[m - x - y];
    }
  }
}

template <int D, int P>
constexpr int ncoef_t() {
  return D == 2 ? (P + 1) * (P + 2) / 2 : (P + 1) * (P + 2) * (P + 3) / 6;
}

__device__ __forceinline__ double mono_eval(const Mono& M, const double* U, const double xi[3]) {
  double pw[3][5];
  for (int a = 0; a < 3; ++a) {
    pw[a][0] = 1.0;
    for (int e = 1; e <= M.p; ++e) pw[a][e] = pw[a][e - 1] * xi[a];
  }
  double s = 0.0;
  for (int al = 0; al < M.n; ++al) {
    double t = U[al];
    for (int a = 0; a < M.d; ++a) t *= pw[a][M.E[al][a]];
    s += t;
  }
  return s;
}

// ---------------------------------------------------------------- kernels
// ctl != null: GMRES iteration on the device; the input is the basis vector
// V[j] with j = ctl[0], and nothing is done once ctl[1] (converged) is set
__global__ void k_extend(int64_t ns, int p, const int* idx, const double* w, const double* psi,
                         double* out, const int* ctl, const double* Vb, int64_t nv) {
  if (ctl) {
    if (ctl[1]) return;
    psi = Vb + (int64_t)ctl[0] * nv;
  }
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  double v = 0.0;
  for (int j = 0; j < p; ++j) {
    int i = idx[s * p + j];
    if (i >= 0) v += w[s * p + j] * psi[i];
  }
  out[s] = v;
}

struct CoefArgs {
  int64_t n_dof;
  int n, nP, nD, nN;
  double h;
  double bscale, fscale;   // b and ftilde enter multiplied by these (1 but for the two-density form)
  const double *MinvT, *MT;
  const double *a, *b, *ftilde;
  const int *stD, *stN;
  double* U;
};

// error-free transformations (Knuth two-sum; product error by fma)
__device__ __forceinline__ void two_sum(double x, double y, double& s, double& e) {
  s = x + y;
  double z = s - x;
  e = (x - (s - z)) + (y - z);
}

// U[c] solves M U = Q, Q = [h^2 ftilde(PDE pts) ; a(D pts) ; h b(N pts)]
// (Sec. 5.3.1, eq. cau-ls): U1 = Minv Q, then one refinement step
// U = U1 + Minv r with the residual r = Q - M U1 summed in compensated
// (twice working) precision, which makes U the rounded exact solution of
// the square system independent of how the inverse was formed.  One
// wavefront per centre, lane = row / coefficient index.
constexpr int COEF_WAVES = KFBI_BLOCK / 64;

__global__ void __launch_bounds__(KFBI_BLOCK) k_coef(CoefArgs a) {
  __shared__ double Qs[COEF_WAVES][KFBI_MAXC], Us[COEF_WAVES][KFBI_MAXC], Rs[COEF_WAVES][KFBI_MAXC];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * COEF_WAVES + wv;
  if (c >= a.n_dof) return;           // whole wavefronts leave together
  const int n = a.n;
  if (lane < n) {
    const int j = lane;
    double q = 0.0;
    if (j < a.nP) {
      if (a.ftilde) q = (a.h * a.h) * (a.fscale * a.ftilde[c * a.nP + j]);
    } else if (j < a.nP + a.nD) {
      if (a.a) q = a.a[a.stD[c * a.nD + (j - a.nP)]];
    } else {
      if (a.b) q = a.h * (a.bscale * a.b[a.stN[c * a.nN + (j - a.nP - a.nD)]]);
    }
    Qs[wv][j] = q;
  }
  __builtin_amdgcn_wave_barrier();
  const double* Mi = a.MinvT + c * (int64_t)n * n;
  if (lane < n) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += Mi[j * n + lane] * Qs[wv][j];
    Us[wv][lane] = s;
  }
  __builtin_amdgcn_wave_barrier();
  if (lane < n) {
    const double* mt = a.MT + c * (int64_t)n * n;
    double s = Qs[wv][lane], comp = 0.0;
    for (int al = 0; al < n; ++al) {
      const double m = mt[al * n + lane], u = Us[wv][al];
      const double p = m * u;
      const double pe = fma(m, u, -p);
      double t, e;
      two_sum(s, -p, t, e);
      s = t;
      comp += e - pe;
    }
    Rs[wv][lane] = s + comp;
  }
  __builtin_amdgcn_wave_barrier();
  if (lane < n) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += Mi[j * n + lane] * Rs[wv][j];
    a.U[c * n + lane] = Us[wv][lane] + s;
  }
}

struct CorrArgs {
  GridDesc g;
  Mono M;
  int64_t n_corr;
  const int *ck, *cnode, *cown, *d2s;
  const double *spos, *U;
  double* Cg;
};

__global__ void k_corr_values(CorrArgs a) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.n_corr) return;
  const GridDesc& g = a.g;
  int c[3];
  int64_t node = a.cnode[e];
  unravel(g, node, c);
  int own = a.cown[e];
  const double* P = a.spos + (int64_t)a.d2s[own] * g.d;
  double xi[3] = {0.0, 0.0, 0.0};
  for (int ax = 0; ax < g.d; ++ax) xi[ax] = ((g.lo + (double)c[ax] * g.h) - P[ax]) / g.h;
  a.Cg[(int64_t)(a.ck[e] - 1) * g.n_nodes + node] = mono_eval(a.M, a.U + (int64_t)own * a.M.n, xi);
}

struct RhsArgs {
  GridDesc g;
  Stencil S;
  const int8_t* region;
  const double *fhat, *gB;
  double* F;
  const double* Cg;   // non-null: the correction of k_rhs_correct is added in the same pass
  int fsel;           // fhat of every region (0), the interiors only (1), the exterior only (2)
};

// F(P) = B_h fhat_{reg P}(P) - sum_{Q on the box boundary} A_PQ gB(Q); with
// Cg, plus at the irregular nodes the correction -sum over cut neighbours Q
// of A_PQ (C^(reg P) - C^(reg Q))(Q), summed as k_rhs_correct sums it
__global__ void k_rhs_base(RhsArgs a) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const GridDesc& g = a.g;
  if (i >= g.n_nodes) return;
  int c[3];
  unravel(g, i, c);
  for (int ax = 0; ax < g.d; ++ax)
    if (c[ax] < 1 || c[ax] > g.N - 1) return;
  int zr = g.d == 3 ? 1 : 0;
  double s = 0.0;
  const int ri = a.region[i];
  const bool fon = a.fsel == 0 || (a.fsel == 1 ? ri != 0 : ri == 0);
  const double* f = a.fhat && fon ? a.fhat + (int64_t)ri * g.n_nodes : nullptr;
  for (int o2 = -zr; o2 <= zr; ++o2)
    for (int o1 = -1; o1 <= 1; ++o1)
      for (int o0 = -1; o0 <= 1; ++o0) {
        int idx = (o0 + 1) + 3 * (o1 + 1) + 9 * (o2 + 1);
        int q0 = c[0] + o0, q1 = c[1] + o1, q2 = c[2] + o2;
        int64_t Q = ravel(g, q0, q1, q2);
        if (f && a.S.B[idx] != 0.0) s += a.S.B[idx] * f[Q];
        if (a.gB && a.S.A[idx] != 0.0) {
          bool bd = q0 == 0 || q0 == g.N || q1 == 0 || q1 == g.N ||
                    (g.d == 3 && (q2 == 0 || q2 == g.N));
          if (bd) s -= a.S.A[idx] * a.gB[Q];
        }
      }
  if (a.Cg) {
    const int rp = a.region[i];
    double corr = 0.0;
    bool cut = false;
    for (int o2 = -zr; o2 <= zr; ++o2)
      for (int o1 = -1; o1 <= 1; ++o1)
        for (int o0 = -1; o0 <= 1; ++o0) {
          const int idx = (o0 + 1) + 3 * (o1 + 1) + 9 * (o2 + 1);
          const double w = a.S.A[idx];
          if (w == 0.0 || (o0 == 0 && o1 == 0 && o2 == 0)) continue;
          const int64_t Q = ravel(g, c[0] + o0, c[1] + o1, c[2] + o2);
          const int rq = a.region[Q];
          if (rq == rp) continue;
          cut = true;
          corr -= w * (Cval(a.Cg, g.n_nodes, rp, Q) - Cval(a.Cg, g.n_nodes, rq, Q));
        }
    if (cut) s = s + corr;
  }
  a.F[i] = s;
}

struct RhsCorrArgs {
  const int* ctl;
  GridDesc g;
  Stencil S;
  int64_t n_irr;
  const int* irr;
  const int8_t* region;
  const double* Cg;
  double* F;
  int overwrite;
};

__global__ void k_rhs_correct(RhsCorrArgs a) {
  if (a.ctl && a.ctl[1]) return;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.n_irr) return;
  const GridDesc& g = a.g;
  int64_t P = a.irr[t];
  int c[3];
  unravel(g, P, c);
  int rp = a.region[P];
  int zr = g.d == 3 ? 1 : 0;
  double corr = 0.0;
  for (int o2 = -zr; o2 <= zr; ++o2)
    for (int o1 = -1; o1 <= 1; ++o1)
      for (int o0 = -1; o0 <= 1; ++o0) {
        int idx = (o0 + 1) + 3 * (o1 + 1) + 9 * (o2 + 1);
        double w = a.S.A[idx];
        if (w == 0.0 || (o0 == 0 && o1 == 0 && o2 == 0)) continue;
        int64_t Q = ravel(g, c[0] + o0, c[1] + o1, c[2] + o2);
        int rq = a.region[Q];
        if (rq == rp) continue;
        corr -= w * (Cval(a.Cg, g.n_nodes, rp, Q) - Cval(a.Cg, g.n_nodes, rq, Q));
      }
  a.F[P] = a.overwrite ? corr : a.F[P] + corr;
}

__global__ void k_boundary(GridDesc g, const double* gB, double* v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n_nodes) return;
  int c[3];
  unravel(g, i, c);
  bool bd = false;
  for (int ax = 0; ax < g.d; ++ax) bd = bd || c[ax] == 0 || c[ax] == g.N;
  if (bd) v[i] = gB ? gB[i] : 0.0;
}

__global__ void k_bie_rhs(GridDesc g, int64_t n_dof, const int* d2s, const double* g2, const double* dn_in,
                          const double* dn_out, double* b) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_dof) return;
  double J = g.beta_in * dn_in[c] - g.beta_out * dn_out[c];
  b[c] = (g2[d2s[c]] - J) / (g.beta_in + g.beta_out);
}


// ---------------------------------------------------------------- folded operators
// At set-up the inverses and the density extension are folded into the
// linear maps the matvec needs (U = Minv Q with Q = [0; 0; h psiS(N pts)];
// for a Dirichlet problem the density is the jump [u], Q = [0; phiS(D pts);
// 0], the maps use the Dirichlet columns without the factor h, and the
// interpolation returns values: IW are the value weights of the block and
// C_c(p_c) = U[0] takes the place of d_n C_c(p_c)):
//   C at entry e        = sum_t FW[e][t] psi[FI[e][t]]
//                         (FW = h phi(xi_e)^T Minv[:, N col j] * extension weight)
//   d_n C_c(p_c)        = sum_t GW[c][t] psi[GI[c][t]]
//                         (GW = sum_a n_a Minv[e_a, N col j] * extension weight)
//   d_n v_in(p_c)       = sum_b IW[c][b] (v(b) - C^(reg b)(b) [b inside another interface])
//                         + sum_t HW[c][t] psi[GI[c][t]]
//                         (the centre's own polynomial at the block nodes outside its
//                          region: TI[c] = sum_b IW[c][b] phi(xi_b) over those nodes,
//                          HW = h TI^T Minv[:, N col j] * extension weight)
// plus the cut-neighbour lists of the irregular nodes and the entries of the
// interpolation blocks, so a matvec is a short chain of gathers.
struct FoldArgs {
  GridDesc g;
  Mono M;
  int nP, nD, nN, nC, nF, maxpairs;
  int64_t n_dof, n_corr, n_irr;
  const int *d2s, *ck, *cnode, *cown, *stD, *stN, *ext_idx, *irr, *EI, *meta;
  const int8_t* region;
  const double *spos, *snrm, *MinvT, *ext_w;
  int *FI, *GI, *IB, *IE2, *PE1, *PE2;
  const int* flags;    // status flags: the folds do nothing when one is set (the tables may be invalid)
  double *FW, *GW, *HW, *IW, *TI, *PA;
  Stencil S;
  // two-density plans: the scale h / sigma of the flux density's columns,
  // and the value-interpolation folds (C_c(p_c) and the own-polynomial term)
  double nscale;
  double *GWv, *HWv;
  const double* TIv;
};

// The density columns of the folds.  Single density: the flux jump in the
// Neumann columns (scale h), or for a Dirichlet problem the value jump in
// the Dirichlet columns (scale 1).  Two-density: group 0 is phi in the
// Dirichlet columns (scale 1, density indices 0..n), group 1 psi in the
// Neumann columns (scale h / sigma of the plan, indices n..2n); their terms
// are stored one after the other (jbase).
struct DenCols {
  int col0, cnt, jbase;
  const int* st;
  double scale;
  int ioff;
};

__device__ __forceinline__ int den_groups(const FoldArgs& a) { return a.g.bie == KFBI_BIE_TWO_DENSITY ? 2 : 1; }

__device__ __forceinline__ DenCols den_cols(const FoldArgs& a, int grp) {
  const bool dir = a.g.bie == KFBI_BIE_DIRICHLET, td = a.g.bie == KFBI_BIE_TWO_DENSITY;
  DenCols c;
  if (dir || (td && grp == 0)) {
    c.col0 = a.nP;
    c.cnt = a.nD;
    c.st = a.stD;
    c.scale = 1.0;
    c.ioff = 0;
    c.jbase = 0;
  } else {
    c.col0 = a.nP + a.nD;
    c.cnt = a.nN;
    c.st = a.stN;
    c.scale = td ? a.nscale : a.g.h;
    c.ioff = td ? (int)a.n_dof : 0;
    c.jbase = td ? a.nD : 0;
  }
  return c;
}

__global__ void k_entry_map(int64_t n_corr, int64_t n_nodes, const int* ck, const int* cnode, int* EI) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_corr) return;
  EI[(int64_t)(ck[e] - 1) * n_nodes + cnode[e]] = (int)e;
}

template <int D, int P>
__global__ void k_fold_corr(FoldArgs a) {
  if (*a.flags) return;
  constexpr int NC = ncoef_t<D, P>();
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.n_corr) return;
  const GridDesc& g = a.g;
  int c[3];
  unravel(g, a.cnode[e], c);
  int own = a.cown[e];
  const double* P0 = a.spos + (int64_t)a.d2s[own] * D;
  double xi[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int ax = 0; ax < D; ++ax) xi[ax] = ((g.lo + (double)c[ax] * g.h) - P0[ax]) / g.h;
  double phi[NC];
  monomials<D, P>(xi, phi);
  const double* Mi = a.MinvT + (int64_t)own * NC * NC;
  for (int grp = 0; grp < den_groups(a); ++grp) {
    const DenCols dc = den_cols(a, grp);
    for (int j = 0; j < dc.cnt; ++j) {
      const double* col = Mi + (int64_t)(dc.col0 + j) * NC;
      double sacc = 0.0;
#pragma unroll
      for (int al = 0; al < NC; ++al) sacc += col[al] * phi[al];
      const double rn = dc.scale * sacc;
      const int sN = dc.st[(int64_t)own * dc.cnt + j];
#pragma unroll
      for (int m = 0; m < P; ++m) {
        const int idx = a.ext_idx[(int64_t)sN * P + m];
        const int64_t o = e * a.nF + (int64_t)(dc.jbase + j) * P + m;
        a.FI[o] = idx >= 0 ? dc.ioff + idx : 0;
        a.FW[o] = idx >= 0 ? rn * a.ext_w[(int64_t)sN * P + m] : 0.0;
      }
    }
  }
}

__global__ void k_fold_dof(FoldArgs a) {
  if (*a.flags) return;
  const GridDesc& g = a.g;
  const int q = g.p, q1 = q + 1;
  const int nbk = g.d == 3 ? q1 * q1 * q1 : q1 * q1;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t c = t / nbk;
  int b = (int)(t % nbk);
  if (c >= a.n_dof) return;
  int s = a.d2s[c];
  const int k = a.meta[(int64_t)s * 5 + 3];
  const double* P = a.spos + (int64_t)s * g.d;
  const double* nv = a.snrm + (int64_t)s * g.d;
  int bb[3] = {b % q1, (b / q1) % q1, b / (q1 * q1)};
  int st[3] = {0, 0, 0};
  double val[3], der[3];
  for (int ax = 0; ax < g.d; ++ax) {
    double tt = (P[ax] - g.lo) / g.h;
    int b0 = (int)floor(tt + 0.5) - q / 2;
    if (b0 < 0) b0 = 0;
    if (b0 > g.N - q) b0 = g.N - q;
    st[ax] = b0;
    double u = tt - (double)b0;
    int j = bb[ax];
    double v = 1.0;
    for (int m = 0; m <= q; ++m)
      if (m != j) v = v * (u - (double)m) / (double)(j - m);
    double dv = 0.0;
    for (int l = 0; l <= q; ++l) {
      if (l == j) continue;
      double w = 1.0 / (double)(j - l);
      for (int m = 0; m <= q; ++m)
        if (m != j && m != l) w = w * (u - (double)m) / (double)(j - m);
      dv += w;
    }
    val[ax] = v;
    der[ax] = dv;
  }
  const bool dir = g.bie == KFBI_BIE_DIRICHLET;
  double w = 0.0;
  if (dir) {
    w = 1.0;
    for (int ax = 0; ax < g.d; ++ax) w = w * val[ax];
  } else {
    for (int ax = 0; ax < g.d; ++ax) {
      double t2 = der[ax] / g.h;
      for (int o = 0; o < g.d; ++o)
        if (o != ax) t2 = t2 * val[o];
      w += nv[ax] * t2;
    }
  }
  a.IW[c * nbk + b] = w;
  // entry of C^(reg q) at a block node inside another interface (-1 elsewhere)
  const int64_t Q = ravel(g, st[0] + bb[0], st[1] + bb[1], st[2] + bb[2]);
  const int rq = a.region[Q];
  a.IE2[c * nbk + b] = (rq != k && rq != 0) ? a.EI[(int64_t)(rq - 1) * g.n_nodes + Q] : -1;
  if (b == 0) {
    a.IB[c] = (int)ravel(g, st[0], st[1], st[2]);
    const double* Mi = a.MinvT + c * (int64_t)a.nC * a.nC;
    const bool td = g.bie == KFBI_BIE_TWO_DENSITY;
    for (int grp = 0; grp < den_groups(a); ++grp) {
      const DenCols dc = den_cols(a, grp);
      for (int j = 0; j < dc.cnt; ++j) {
        const double* col = Mi + (int64_t)(dc.col0 + j) * a.nC;
        double gsum = 0.0;
        if (dir)
          gsum = col[0];                                                   // C_c(p_c) = U[0]
        else
          for (int ax = 0; ax < g.d; ++ax) gsum += nv[ax] * col[1 + ax];   // graded order: 1, x, y(, z)
        // two-density: d_n C_c(p_c) = U[1 + ax] n_ax / h with U = scale Minv Q
        if (td) gsum = gsum * (dc.scale / g.h);
        const int sN = dc.st[c * dc.cnt + j];
        for (int m = 0; m < g.p; ++m) {
          const int idx = a.ext_idx[(int64_t)sN * g.p + m];
          const int64_t o = c * a.nF + (int64_t)(dc.jbase + j) * g.p + m;
          const double ew = idx >= 0 ? a.ext_w[(int64_t)sN * g.p + m] : 0.0;
          a.GI[o] = idx >= 0 ? dc.ioff + idx : 0;
          a.GW[o] = idx >= 0 ? gsum * ew : 0.0;
          if (td) a.GWv[o] = idx >= 0 ? (col[0] * dc.scale) * ew : 0.0;
        }
      }
    }
  }
}

// the centre's own polynomial in its interpolation: TI[c] = sum over the
// block nodes outside the centre's region of IW * monomials(xi_b), and its
// fold HW with the Neumann columns of the inverse and the extension.  A
// group of FOLD_G lanes per centre: the lanes split the block nodes, the
// partial sums of T are combined by a fixed butterfly, and the lanes then
// split the nN * P folded weights.
constexpr int FOLD_G = 32;

// HW[c][t] (or HWv) = scale T . Minv[:, column] * extension weight over the
// density columns; the lanes of the centre's group split the terms
template <int NC, int P>
__device__ __forceinline__ void fold_own_terms(const FoldArgs& a, int64_t c, int lane, const double* T, double* out) {
  const double* Mi = a.MinvT + c * (int64_t)NC * NC;
  const DenCols d0 = den_cols(a, 0);
  const int n0 = d0.cnt * P;
  const int tot = den_groups(a) == 2 ? n0 + a.nN * P : n0;
  for (int q = lane; q < tot; q += FOLD_G) {
    const DenCols dc = q < n0 ? d0 : den_cols(a, 1);
    const int qq = q < n0 ? q : q - n0;
    const int j = qq / P, m = qq % P;
    const double* col = Mi + (int64_t)(dc.col0 + j) * NC;
    double sacc = 0.0;
#pragma unroll
    for (int al = 0; al < NC; ++al) sacc += T[al] * col[al];
    const double rn = dc.scale * sacc;
    const int sN = dc.st[c * dc.cnt + j];
    const int idx = a.ext_idx[(int64_t)sN * P + m];
    out[c * a.nF + (int64_t)(dc.jbase + j) * P + m] = idx >= 0 ? rn * a.ext_w[(int64_t)sN * P + m] : 0.0;
  }
}

template <int D, int P>
__global__ void __launch_bounds__(KFBI_BLOCK) k_fold_own(FoldArgs a) {
  if (*a.flags) return;
  constexpr int NC = ncoef_t<D, P>();
  constexpr int Q1 = P + 1;
  constexpr int NBK = D == 3 ? Q1 * Q1 * Q1 : Q1 * Q1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = t / FOLD_G;
  const int lane = (int)(t % FOLD_G);
  if (c >= a.n_dof) return;   // whole groups leave together
  const GridDesc& g = a.g;
  const int s = a.d2s[c];
  const int k = a.meta[(int64_t)s * 5 + 3];
  const double* P0 = a.spos + (int64_t)s * D;
  const int64_t base = a.IB[c];
  int st[3] = {0, 0, 0};
  unravel(g, base, st);
  double T[NC];
#pragma unroll
  for (int al = 0; al < NC; ++al) T[al] = 0.0;
  for (int b = lane; b < NBK; b += FOLD_G) {
    const int bb[3] = {b % Q1, (b / Q1) % Q1, b / (Q1 * Q1)};
    const int64_t Q = ravel(g, st[0] + bb[0], st[1] + bb[1], st[2] + bb[2]);
    if (a.region[Q] == k) continue;
    double xi[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int ax = 0; ax < D; ++ax) xi[ax] = ((g.lo + (double)(st[ax] + bb[ax]) * g.h) - P0[ax]) / g.h;
    double phi[NC];
    monomials<D, P>(xi, phi);
    const double w = a.IW[c * NBK + b];
#pragma unroll
    for (int al = 0; al < NC; ++al) T[al] += w * phi[al];
  }
#pragma unroll
  for (int off = FOLD_G / 2; off > 0; off >>= 1) {
#pragma unroll
    for (int al = 0; al < NC; ++al) T[al] += __shfl_xor(T[al], off, FOLD_G);
  }
  if (lane == 0) {
#pragma unroll
    for (int al = 0; al < NC; ++al) a.TI[c * NC + al] = T[al];
  }
  fold_own_terms<NC, P>(a, c, lane, T, a.HW);
}

// the own-polynomial fold of the value interpolation (two-density plans):
// the same terms with TIv
template <int D, int P>
__global__ void __launch_bounds__(KFBI_BLOCK) k_fold_hwv(FoldArgs a) {
  if (*a.flags) return;
  constexpr int NC = ncoef_t<D, P>();
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = t / FOLD_G;
  const int lane = (int)(t % FOLD_G);
  if (c >= a.n_dof) return;
  double T[NC];
#pragma unroll
  for (int al = 0; al < NC; ++al) T[al] = a.TIv[c * NC + al];
  fold_own_terms<NC, P>(a, c, lane, T, a.HWv);
}

// cut neighbours of every irregular node: stencil coefficient and the
// entries of C^(reg P) and C^(reg Q) at the neighbour (Sec. 5.2 remark)
__global__ void k_fold_pairs(FoldArgs a) {
  if (*a.flags) return;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.n_irr) return;
  const GridDesc& g = a.g;
  int64_t P = a.irr[t];
  int c[3];
  unravel(g, P, c);
  int rp = a.region[P];
  int zr = g.d == 3 ? 1 : 0;
  int m = 0;
  for (int o2 = -zr; o2 <= zr; ++o2)
    for (int o1 = -1; o1 <= 1; ++o1)
      for (int o0 = -1; o0 <= 1; ++o0) {
        int idx = (o0 + 1) + 3 * (o1 + 1) + 9 * (o2 + 1);
        double w = a.S.A[idx];
        if (w == 0.0 || (o0 == 0 && o1 == 0 && o2 == 0)) continue;
        int64_t Q = ravel(g, c[0] + o0, c[1] + o1, c[2] + o2);
        int rq = a.region[Q];
        if (rq == rp) continue;
        a.PA[t * a.maxpairs + m] = w;
        a.PE1[t * a.maxpairs + m] = rp ? a.EI[(int64_t)(rp - 1) * g.n_nodes + Q] : -1;
        a.PE2[t * a.maxpairs + m] = rq ? a.EI[(int64_t)(rq - 1) * g.n_nodes + Q] : -1;
        ++m;
      }
  for (; m < a.maxpairs; ++m) {
    a.PA[t * a.maxpairs + m] = 0.0;
    a.PE1[t * a.maxpairs + m] = -1;
    a.PE2[t * a.maxpairs + m] = -1;
  }
}

__global__ void k_irr_rows(int64_t n_irr, int n1, const int* irr, int* rs, int* re) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_irr) return;
  int row = irr[t] / n1;
  int prev = t > 0 ? irr[t - 1] / n1 : -1;
  int next = t + 1 < n_irr ? irr[t + 1] / n1 : -1;
  if (prev != row) rs[row] = (int)t;
  if (next != row) re[row] = (int)(t + 1);
}

// correction values of all entries: C(e) = sum_t FW[e][t] psi[FI[e][t]],
// G lanes per entry
template <int G>
__global__ void __launch_bounds__(KFBI_BLOCK) k_centry(int64_t n_corr, int nF, const int* FI, const double* FW,
                                                      const double* psi, double* Cv, const int* ctl,
                                                      const double* Vb, int64_t n_dof) {
  // the iteration state is read first and used only after the entry's
  // first index / weight loads are issued (they do not depend on it)
  int stop = 0;
  int64_t jv = 0;
  if (ctl) {
    stop = ctl[1];
    jv = ctl[0];
  }
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t e = t / G;
  int lane = (int)(t % G);
  if (e >= n_corr) return;
  constexpr int PRE = 2;
  int fi[PRE];
  double fw[PRE];
#pragma unroll
  for (int u = 0; u < PRE; ++u) {
    const int q = lane + u * G;
    fi[u] = q < nF ? FI[e * nF + q] : 0;
    fw[u] = q < nF ? FW[e * nF + q] : 0.0;
  }
  if (stop) return;
  if (ctl) psi = Vb + jv * n_dof;
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < PRE; ++u)
    if (lane + u * G < nF) s += fw[u] * psi[fi[u]];
  for (int q = lane + PRE * G; q < nF; q += G) s += FW[e * nF + q] * psi[FI[e * nF + q]];
  for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, G);
  if (lane == 0) Cv[e] = s;
}

// F at every irregular node from the correction values of the current
// density: F = -sum over the node's cut neighbours Q of A_PQ (C^(reg P) -
// C^(reg Q))(x_Q).  One group of 32 lanes per node, lane m takes pair m
// (up to 26 in 3D), the group sum is a fixed butterfly; used where the pair
// table is long (3D, 4th order), so that the first box-solve pass reads one
// value per irregular node instead of walking the pairs.
constexpr int IRR_G = 32;
__global__ void __launch_bounds__(KFBI_BLOCK) k_irr_rhs(int64_t n_irr, int maxpairs, const double* PA, const int* PE1,
                                                       const int* PE2, const double* Cv, double* Firr,
                                                       const int* ctl) {
  if (ctl && ctl[1]) return;
  const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / IRR_G;
  const int m = (int)(threadIdx.x % IRR_G);
  if (t >= n_irr) return;   // whole groups leave together
  double v = 0.0;
  if (m < maxpairs) {
    const int64_t o = t * maxpairs + m;
    const double cf = PA[o];
    if (cf != 0.0) {
      const int e1 = PE1[o], e2 = PE2[o];
      const double c1 = e1 >= 0 ? Cv[e1] : 0.0, c2 = e2 >= 0 ? Cv[e2] : 0.0;
      v = cf * (c1 - c2);
    }
  }
  for (int off = IRR_G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, IRR_G);
  if (m == 0) Firr[t] = -v;
}

struct InterpArgs {
  const int* ctl;        // GMRES iteration on the device: psi = V[j], output V[j + 1], j = ctl[0]
  double* Vb;
  GridDesc g;
  int nbk, nC, nF;
  int64_t n_dof;
  const int *d2s, *meta, *IB;
  const double *IW, *U, *snrm, *v, *Cg;
  // folded matvec path (U == null)
  const int *IE2, *GI;
  const double *Cv, *GW, *HW, *TI, *psi;
  const int8_t* region;
  double *dn_in, *dn_out, *Apsi;
  int value;             // 1: one-sided values (IW value weights, C_{h,p}(p) = U[0]); 0: normal derivatives
};

// one group of G lanes per centre: sum_b IW[c][b] vtilde(b), then the combine
template <int G>
__global__ void __launch_bounds__(KFBI_BLOCK) k_interp(InterpArgs a) {
  // the iteration state is read first and used only after the box-solution
  // sum (which does not depend on it) has its loads in flight
  int stop = 0;
  int64_t jv = 0;
  if (a.ctl) {
    stop = a.ctl[1];
    jv = a.ctl[0];
  }
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t c = t / G;
  int lane = (int)(t % G);
  if (c >= a.n_dof) return;           // whole groups leave together
  const GridDesc& g = a.g;
  const int q1 = g.p + 1;
  const int s = a.d2s[c];
  const int k = a.meta[(int64_t)s * 5 + 3];
  const int64_t base = a.IB[c];
  const double* w = a.IW + c * a.nbk;
  double acc = 0.0;
  for (int b = lane; b < a.nbk; b += G) {
    int b0 = b % q1, b1 = (b / q1) % q1, b2 = b / (q1 * q1);
    int64_t Q = base + b0 + (int64_t)g.n1 * (b1 + (int64_t)g.n1 * b2);
    double vt = a.v[Q];
    if (a.U) {
      int rq = a.region[Q];
      if (rq != k && rq != 0) vt -= Cval(a.Cg, g.n_nodes, rq, Q);
    } else {
      const int e2 = a.IE2[c * a.nbk + b];
      if (e2 >= 0) vt -= a.Cv[e2];
    }
    acc += w[b] * vt;
  }
  if (stop) return;
  if (a.ctl) {
    a.psi = a.Vb + jv * a.n_dof;
    a.Apsi = a.Vb + (jv + 1) * a.n_dof;
  }
  // the centre's own polynomial at the block nodes outside its region
  double dnC = 0.0;
  if (!a.U) {
    for (int q = lane; q < a.nF; q += G) {
      const double ps = a.psi[a.GI[c * a.nF + q]];
      dnC += a.GW[c * a.nF + q] * ps;
      acc += a.HW[c * a.nF + q] * ps;
    }
  } else {
    for (int al = lane; al < a.nC; al += G) acc += a.TI[c * a.nC + al] * a.U[c * (int64_t)a.nC + al];
  }
  for (int off = G / 2; off > 0; off >>= 1) {
    acc += __shfl_xor(acc, off, G);
    dnC += __shfl_xor(dnC, off, G);
  }
  if (lane != 0) return;
  if (a.U) {
    const double* Uc = a.U + c * (int64_t)a.nC;
    if (a.value) {
      dnC = Uc[0];   // value trace: the jump C_{h,p}(p)
    } else {
      const double* nv = a.snrm + (int64_t)s * g.d;
      for (int ax = 0; ax < g.d; ++ax) dnC += nv[ax] * Uc[1 + ax];
      dnC = dnC / g.h;
    }
  }
  double dout = acc - dnC;
  if (a.dn_in) a.dn_in[c] = acc;
  if (a.dn_out) a.dn_out[c] = dout;
  if (a.Apsi) a.Apsi[c] = (g.beta_in * acc - g.beta_out * dout) / (g.beta_in + g.beta_out);
}

// Value weights of the interpolation blocks, for plans that need both
// one-sided values and normal derivatives (the two-density BIE): IWv[c][b]
// = prod_ax L_{b_ax}(t_ax), the tensor Lagrange basis of the block at the
// centre (Sec. 5.5), in the order the value weights of a Dirichlet plan use.
__global__ void k_fold_values(GridDesc g, int64_t n_dof, const int* d2s, const double* spos, const int* flags,
                              double* IWv) {
  if (*flags) return;
  const int q = g.p, q1 = q + 1;
  const int nbk = g.d == 3 ? q1 * q1 * q1 : q1 * q1;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t c = t / nbk;
  int b = (int)(t % nbk);
  if (c >= n_dof) return;
  const double* P = spos + (int64_t)d2s[c] * g.d;
  int bb[3] = {b % q1, (b / q1) % q1, b / (q1 * q1)};
  double w = 1.0;
  for (int ax = 0; ax < g.d; ++ax) {
    double tt = (P[ax] - g.lo) / g.h;
    int b0 = (int)floor(tt + 0.5) - q / 2;
    if (b0 < 0) b0 = 0;
    if (b0 > g.N - q) b0 = g.N - q;
    double u = tt - (double)b0;
    int j = bb[ax];
    double v = 1.0;
    for (int m = 0; m <= q; ++m)
      if (m != j) v = v * (u - (double)m) / (double)(j - m);
    w = w * v;
  }
  IWv[c * nbk + b] = w;
}

// TIv[c] = sum over the block nodes outside the centre's region of IWv *
// monomials(xi_b): the centre's own polynomial in its value interpolation
template <int D, int P>
__global__ void __launch_bounds__(KFBI_BLOCK) k_fold_tiv(FoldArgs a, const double* IWv, double* TIv) {
  if (*a.flags) return;
  constexpr int NC = ncoef_t<D, P>();
  constexpr int Q1 = P + 1;
  constexpr int NBK = D == 3 ? Q1 * Q1 * Q1 : Q1 * Q1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = t / FOLD_G;
  const int lane = (int)(t % FOLD_G);
  if (c >= a.n_dof) return;   // whole groups leave together
  const GridDesc& g = a.g;
  const int s = a.d2s[c];
  const int k = a.meta[(int64_t)s * 5 + 3];
  const double* P0 = a.spos + (int64_t)s * D;
  int st[3] = {0, 0, 0};
  unravel(g, a.IB[c], st);
  double T[NC];
#pragma unroll
  for (int al = 0; al < NC; ++al) T[al] = 0.0;
  for (int b = lane; b < NBK; b += FOLD_G) {
    const int bb[3] = {b % Q1, (b / Q1) % Q1, b / (Q1 * Q1)};
    const int64_t Q = ravel(g, st[0] + bb[0], st[1] + bb[1], st[2] + bb[2]);
    if (a.region[Q] == k) continue;
    double xi[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int ax = 0; ax < D; ++ax) xi[ax] = ((g.lo + (double)(st[ax] + bb[ax]) * g.h) - P0[ax]) / g.h;
    double phi[NC];
    monomials<D, P>(xi, phi);
    const double w = IWv[c * NBK + b];
#pragma unroll
    for (int al = 0; al < NC; ++al) T[al] += w * phi[al];
  }
#pragma unroll
  for (int off = FOLD_G / 2; off > 0; off >>= 1) {
#pragma unroll
    for (int al = 0; al < NC; ++al) T[al] += __shfl_xor(T[al], off, FOLD_G);
  }
  if (lane == 0) {
#pragma unroll
    for (int al = 0; al < NC; ++al) TIv[c * NC + al] = T[al];
  }
}

// Zero-mean shift of a Neumann problem with kappa = 0 (Sec. 6.2.1): one
// work group sums x in a fixed order and subtracts the mean.  With ctl, x is
// the GMRES basis vector V[j + 1], j = ctl[0].
constexpr int ZM_BLOCK = 1024;
__global__ void __launch_bounds__(ZM_BLOCK) k_zero_mean(int64_t n, double* x, const int* ctl, double* Vb) {
  if (ctl) {
    if (ctl[1]) return;
    x = Vb + ((int64_t)ctl[0] + 1) * n;
  }
  __shared__ double red[ZM_BLOCK];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += ZM_BLOCK) s += x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = ZM_BLOCK / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  const double mean = red[0] / (double)n;
  for (int64_t i = threadIdx.x; i < n; i += ZM_BLOCK) x[i] -= mean;
}

}  // namespace

// ---------------------------------------------------------------- launchers
void op_extend(kfbi_plan* pl, const double* psi, double* psiS) {
  hipLaunchKernelGGL(k_extend, dim3(nb(pl->n_surf)), dim3(KFBI_BLOCK), 0, pl->stream, pl->n_surf, pl->g.p,
                     pl->ext_idx, pl->ext_w, psi, psiS, pl->ctl_active, pl->V, pl->n_dof);
}

void op_coefficients(kfbi_plan* pl, const double* a, const double* b, const double* ftilde, double bscale,
                     double fscale) {
  CoefArgs A{pl->n_dof, pl->nC, pl->nP, pl->nD, pl->nN, pl->g.h, bscale, fscale, pl->MinvT, pl->MT, a, b, ftilde,
             pl->stD, pl->stN, pl->U};
  unsigned blocks = (unsigned)((pl->n_dof + COEF_WAVES - 1) / COEF_WAVES);
  hipLaunchKernelGGL(k_coef, dim3(blocks), dim3(KFBI_BLOCK), 0, pl->stream, A);
}

void op_correction_values(kfbi_plan* pl) {
  if (pl->n_corr == 0) return;
  CorrArgs A{pl->g, make_mono(pl), pl->n_corr, pl->ce_k, pl->ce_node, pl->ce_owner, pl->d2s, pl->s_pos, pl->U,
             pl->Cg};
  hipLaunchKernelGGL(k_corr_values, dim3(nb(pl->n_corr)), dim3(KFBI_BLOCK), 0, pl->stream, A);
}

void op_rhs_base(kfbi_plan* pl, const double* fhat, const double* gB, double* F, bool corrected, int fsel) {
  RhsArgs A{pl->g, make_stencil(pl->g), pl->region, fhat, gB, F, corrected && pl->n_irr > 0 ? pl->Cg : nullptr,
            fsel};
  hipLaunchKernelGGL(k_rhs_base, dim3(nb(pl->g.n_nodes)), dim3(KFBI_BLOCK), 0, pl->stream, A);
}

void op_rhs_correct(kfbi_plan* pl, double* F, bool overwrite) {
  if (pl->n_irr == 0) return;
  RhsCorrArgs A{pl->ctl_active, pl->g, make_stencil(pl->g), pl->n_irr, pl->irr, pl->region, pl->Cg, F,
                overwrite ? 1 : 0};
  hipLaunchKernelGGL(k_rhs_correct, dim3(nb(pl->n_irr)), dim3(KFBI_BLOCK), 0, pl->stream, A);
}

void op_boundary(kfbi_plan* pl, const double* gB, double* v) {
  hipLaunchKernelGGL(k_boundary, dim3(nb(pl->g.n_nodes)), dim3(KFBI_BLOCK), 0, pl->stream, pl->g, gB, v);
}

namespace {
void launch_interp(kfbi_plan* pl, const double* v, const double* U, const double* psi, double* dn_in,
                   double* dn_out, double* Apsi, bool values = false) {
  const int q1 = pl->g.p + 1;
  InterpArgs A;
  A.value = values || pl->g.bie == KFBI_BIE_DIRICHLET ? 1 : 0;
  A.ctl = pl->ctl_active;
  A.Vb = pl->V;
  A.g = pl->g;
  A.nbk = pl->g.d == 3 ? q1 * q1 * q1 : q1 * q1;
  A.nC = pl->nC;
  A.nF = pl->nF;
  A.n_dof = pl->n_dof;
  A.d2s = pl->d2s;
  A.meta = pl->s_meta;
  A.IB = pl->IB;
  A.IW = values ? pl->IWv : pl->IW;
  A.U = U;
  A.snrm = pl->s_nrm;
  A.v = v;
  A.Cg = pl->Cg;
  A.IE2 = pl->IE2;
  A.GI = pl->GI;
  A.Cv = pl->Cv;
  A.GW = values ? pl->GWv : pl->GW;
  A.HW = values ? pl->HWv : pl->HW;
  A.TI = values ? pl->TIv : pl->TI;
  A.psi = psi;
  A.region = pl->region;
  A.dn_in = dn_in;
  A.dn_out = dn_out;
  A.Apsi = Apsi;
  if (pl->g.d == 3)
    hipLaunchKernelGGL(k_interp<64>, dim3(nb(pl->n_dof * 64)), dim3(KFBI_BLOCK), 0, pl->stream, A);
  else if (q1 == 5)
    hipLaunchKernelGGL(k_interp<32>, dim3(nb(pl->n_dof * 32)), dim3(KFBI_BLOCK), 0, pl->stream, A);
  else
    hipLaunchKernelGGL(k_interp<16>, dim3(nb(pl->n_dof * 16)), dim3(KFBI_BLOCK), 0, pl->stream, A);
}
}  // namespace

void op_normal_derivatives(kfbi_plan* pl, const double* v, double* dn_in, double* dn_out, double* Apsi) {
  launch_interp(pl, v, pl->U, nullptr, dn_in, dn_out, Apsi);
}

void op_values(kfbi_plan* pl, const double* v, double* v_in, double* v_out) {
  launch_interp(pl, v, pl->U, nullptr, v_in, v_out, nullptr, true);
}

void op_interp_folded(kfbi_plan* pl, const double* v, const double* x, double* t_in, double* t_out, bool values) {
  launch_interp(pl, v, nullptr, x, t_in, t_out, nullptr, values);
}

template <class T>
static kfbi_status regrow(T** p, int64_t n) {
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

kfbi_status op_fold(kfbi_plan* pl) {
  const GridDesc& g = pl->g;
  const int q1 = g.p + 1;
  const int nbk = g.d == 3 ? q1 * q1 * q1 : q1 * q1;
  pl->nF = (g.bie == KFBI_BIE_DIRICHLET ? pl->nD : g.bie == KFBI_BIE_TWO_DENSITY ? pl->nD + pl->nN : pl->nN) * g.p;
  pl->maxpairs = g.order == 2 ? 2 * g.d : (g.d == 3 ? 26 : 8);
  if (pl->n_corr > pl->cap_fold_corr) {
    int64_t cap = kfbi_headroom(pl->n_corr);
    pl->cap_fold_corr = 0;
    KCHK(regrow(&pl->FI, cap * pl->nF));
    KCHK(regrow(&pl->FW, cap * pl->nF));
    KCHK(regrow(&pl->Cv, cap));
    pl->cap_fold_corr = cap;
  }
  if (pl->n_dof > pl->cap_fold_dof) {
    int64_t cap = kfbi_headroom(pl->n_dof);
    pl->cap_fold_dof = 0;
    KCHK(regrow(&pl->GI, cap * pl->nF));
    KCHK(regrow(&pl->GW, cap * pl->nF));
    KCHK(regrow(&pl->HW, cap * pl->nF));
    KCHK(regrow(&pl->TI, cap * pl->nC));
    KCHK(regrow(&pl->IW, cap * nbk));
    KCHK(regrow(&pl->IE2, cap * nbk));
    KCHK(regrow(&pl->IB, cap));
    if (g.bie == KFBI_BIE_TWO_DENSITY) {
      KCHK(regrow(&pl->IWv, cap * nbk));
      KCHK(regrow(&pl->TIv, cap * pl->nC));
      KCHK(regrow(&pl->GWv, cap * pl->nF));
      KCHK(regrow(&pl->HWv, cap * pl->nF));
    }
    pl->cap_fold_dof = cap;
  }
  if (pl->n_irr > pl->cap_fold_irr) {
    int64_t cap = kfbi_headroom(pl->n_irr);
    pl->cap_fold_irr = 0;
    KCHK(regrow(&pl->PA, cap * pl->maxpairs));
    KCHK(regrow(&pl->PE1, cap * pl->maxpairs));
    KCHK(regrow(&pl->PE2, cap * pl->maxpairs));
    KCHK(regrow(&pl->Firr, cap));
    pl->cap_fold_irr = cap;
  }
  // EI (all -1), row_start and row_end (all 0) were cleared at the start of
  // the geometry set-up
  if (pl->n_corr > 0)
    hipLaunchKernelGGL(k_entry_map, dim3(nb(pl->n_corr)), dim3(KFBI_BLOCK), 0, pl->stream, pl->n_corr, g.n_nodes,
                       pl->ce_k, pl->ce_node, pl->EI);
  FoldArgs A;
  A.g = g;
  A.M = make_mono(pl);
  A.nP = pl->nP;
  A.nD = pl->nD;
  A.nN = pl->nN;
  A.nC = pl->nC;
  A.nF = pl->nF;
  A.maxpairs = pl->maxpairs;
  A.n_dof = pl->n_dof;
  A.n_corr = pl->n_corr;
  A.n_irr = pl->n_irr;
  A.d2s = pl->d2s;
  A.ck = pl->ce_k;
  A.cnode = pl->ce_node;
  A.cown = pl->ce_owner;
  A.stD = pl->stD;
  A.stN = pl->stN;
  A.ext_idx = pl->ext_idx;
  A.irr = pl->irr;
  A.EI = pl->EI;
  A.meta = pl->s_meta;
  A.region = pl->region;
  A.spos = pl->s_pos;
  A.snrm = pl->s_nrm;
  A.MinvT = pl->MinvT;
  A.ext_w = pl->ext_w;
  A.FI = pl->FI;
  A.GI = pl->GI;
  A.IB = pl->IB;
  A.IE2 = pl->IE2;
  A.PE1 = pl->PE1;
  A.PE2 = pl->PE2;
  A.FW = pl->FW;
  A.GW = pl->GW;
  A.HW = pl->HW;
  A.IW = pl->IW;
  A.TI = pl->TI;
  A.PA = pl->PA;
  A.S = make_stencil(g);
  A.flags = pl->d_flags;
  A.nscale = g.h / (pl->is_aux ? pl->prob.beta_out : pl->prob.beta_in);
  A.GWv = pl->GWv;
  A.HWv = pl->HWv;
  A.TIv = pl->TIv;
  if (pl->n_corr > 0) {
    dim3 gr(nb(pl->n_corr)), bl(KFBI_BLOCK);
    if (g.d == 2 && g.p == 2) hipLaunchKernelGGL((k_fold_corr<2, 2>), gr, bl, 0, pl->stream, A);
    if (g.d == 2 && g.p == 4) hipLaunchKernelGGL((k_fold_corr<2, 4>), gr, bl, 0, pl->stream, A);
    if (g.d == 3 && g.p == 2) hipLaunchKernelGGL((k_fold_corr<3, 2>), gr, bl, 0, pl->stream, A);
    if (g.d == 3 && g.p == 4) hipLaunchKernelGGL((k_fold_corr<3, 4>), gr, bl, 0, pl->stream, A);
  }
  hipLaunchKernelGGL(k_fold_dof, dim3(nb(pl->n_dof * nbk)), dim3(KFBI_BLOCK), 0, pl->stream, A);
  {
    dim3 gr(nb(pl->n_dof * FOLD_G)), bl(KFBI_BLOCK);
    if (g.d == 2 && g.p == 2) hipLaunchKernelGGL((k_fold_own<2, 2>), gr, bl, 0, pl->stream, A);
    if (g.d == 2 && g.p == 4) hipLaunchKernelGGL((k_fold_own<2, 4>), gr, bl, 0, pl->stream, A);
    if (g.d == 3 && g.p == 2) hipLaunchKernelGGL((k_fold_own<3, 2>), gr, bl, 0, pl->stream, A);
    if (g.d == 3 && g.p == 4) hipLaunchKernelGGL((k_fold_own<3, 4>), gr, bl, 0, pl->stream, A);
  }
  if (g.bie == KFBI_BIE_TWO_DENSITY) {
    hipLaunchKernelGGL(k_fold_values, dim3(nb(pl->n_dof * nbk)), dim3(KFBI_BLOCK), 0, pl->stream, g, pl->n_dof,
                       pl->d2s, pl->s_pos, pl->d_flags, pl->IWv);
    dim3 gr(nb(pl->n_dof * FOLD_G)), bl(KFBI_BLOCK);
    if (g.d == 2 && g.p == 2) hipLaunchKernelGGL((k_fold_tiv<2, 2>), gr, bl, 0, pl->stream, A, pl->IWv, pl->TIv);
    if (g.d == 2 && g.p == 4) hipLaunchKernelGGL((k_fold_tiv<2, 4>), gr, bl, 0, pl->stream, A, pl->IWv, pl->TIv);
    if (g.d == 3 && g.p == 2) hipLaunchKernelGGL((k_fold_tiv<3, 2>), gr, bl, 0, pl->stream, A, pl->IWv, pl->TIv);
    if (g.d == 3 && g.p == 4) hipLaunchKernelGGL((k_fold_tiv<3, 4>), gr, bl, 0, pl->stream, A, pl->IWv, pl->TIv);
    if (g.d == 2 && g.p == 2) hipLaunchKernelGGL((k_fold_hwv<2, 2>), gr, bl, 0, pl->stream, A);
    if (g.d == 2 && g.p == 4) hipLaunchKernelGGL((k_fold_hwv<2, 4>), gr, bl, 0, pl->stream, A);
    if (g.d == 3 && g.p == 2) hipLaunchKernelGGL((k_fold_hwv<3, 2>), gr, bl, 0, pl->stream, A);
    if (g.d == 3 && g.p == 4) hipLaunchKernelGGL((k_fold_hwv<3, 4>), gr, bl, 0, pl->stream, A);
  }
  if (pl->n_irr > 0) {
    hipLaunchKernelGGL(k_fold_pairs, dim3(nb(pl->n_irr)), dim3(KFBI_BLOCK), 0, pl->stream, A);
    hipLaunchKernelGGL(k_irr_rows, dim3(nb(pl->n_irr)), dim3(KFBI_BLOCK), 0, pl->stream, pl->n_irr, g.n1, pl->irr,
                       pl->row_start, pl->row_end);
  }
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

void kfbi_stencil_A(const GridDesc& g, double* A27) {
  Stencil S = make_stencil(g);
  for (int i = 0; i < 27; ++i) A27[i] = S.A[i];
}

// the BIE operator (S2-S5) with the folded maps: the corrected right-hand
// side is formed inside the first box-solve pass, the correction values
// inside the interpolation
void op_matvec(kfbi_plan* pl, const double* psi, double* Apsi) {
  op_matvec_head(pl, psi);
  if (pl->box_solver == KFBI_BOX_FFT) {
    dst_solve_corrections(pl, psi, pl->vbuf);
  } else {
    mg_matvec_rhs(pl);
    mg_solve(pl, pl->Fmg, pl->vbuf);
  }
  op_matvec_tail(pl, psi, Apsi);
}

// the matvec's steps before its box solve: correction values of the
// density (and, FFT, the corrected right-hand side at the irregular nodes
// when its pair lists are long)
void op_matvec_head(kfbi_plan* pl, const double* psi) {
  if (pl->n_corr > 0)
    hipLaunchKernelGGL(k_centry<16>, dim3(nb(pl->n_corr * 16)), dim3(KFBI_BLOCK), 0, pl->stream, pl->n_corr,
                       pl->nF, pl->FI, pl->FW, psi, pl->Cv, pl->ctl_active, pl->V, pl->n_dof);
  if (pl->box_solver == KFBI_BOX_FFT && kfbi_irr_rhs_used(pl) && pl->n_irr > 0)
    hipLaunchKernelGGL(k_irr_rhs, dim3(nb(pl->n_irr * IRR_G)), dim3(KFBI_BLOCK), 0, pl->stream, pl->n_irr,
                       pl->maxpairs, pl->PA, pl->PE1, pl->PE2, pl->Cv, pl->Firr, pl->ctl_active);
}

// after the box solve: the corrected interpolation and the combination
void op_matvec_tail(kfbi_plan* pl, const double* psi, double* Apsi) {
  launch_interp(pl, pl->vbuf, nullptr, psi, nullptr, nullptr, Apsi);
  if (op_zero_mean_used(pl))
    hipLaunchKernelGGL(k_zero_mean, dim3(1), dim3(ZM_BLOCK), 0, pl->stream, pl->n_dof, Apsi, pl->ctl_active, pl->V);
}

void op_bie_rhs(kfbi_plan* pl, const double* g2, const double* dn_in, const double* dn_out, double* b) {
  hipLaunchKernelGGL(k_bie_rhs, dim3(nb(pl->n_dof)), dim3(KFBI_BLOCK), 0, pl->stream, pl->g, pl->n_dof, pl->d2s,
                     g2, dn_in, dn_out, b);
  if (op_zero_mean_used(pl))
    hipLaunchKernelGGL(k_zero_mean, dim3(1), dim3(ZM_BLOCK), 0, pl->stream, pl->n_dof, b, nullptr, nullptr);
}

bool op_zero_mean_used(const kfbi_plan* pl) {
  return pl->g.bie == KFBI_BIE_NEUMANN && pl->g.kappa == 0.0 && pl->n_dof > 0;
}
