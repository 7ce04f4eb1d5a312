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
__global__ void k_extend(int64_t ns, int p, const int* idx, const double* w, const double* psi,
                         double* out) {
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
  const double* MinvT;
  const double *a, *b, *ftilde;
  const int *stD, *stN;
  double* U;
};

// U[c][alpha] = sum_j Minv[c][alpha][j] Q[c][j],
// Q = [h^2 ftilde(PDE pts) ; a(D pts) ; h b(N pts)]   (Sec. 5.3.1, eq. cau-ls)
__global__ void k_coef(CoefArgs a) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t c = t / a.n;
  int al = (int)(t % a.n);
  if (c >= a.n_dof) return;
  const double* Mi = a.MinvT + c * (int64_t)a.n * a.n;
  double s = 0.0;
  if (a.ftilde) {
    double h2 = a.h * a.h;
    for (int j = 0; j < a.nP; ++j) s += Mi[j * a.n + al] * (h2 * a.ftilde[c * a.nP + j]);
  }
  if (a.a)
    for (int j = 0; j < a.nD; ++j) s += Mi[(a.nP + j) * a.n + al] * a.a[a.stD[c * a.nD + j]];
  if (a.b)
    for (int j = 0; j < a.nN; ++j)
      s += Mi[(a.nP + a.nD + j) * a.n + al] * (a.h * a.b[a.stN[c * a.nN + j]]);
  a.U[c * a.n + al] = s;
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
};

// F(P) = B_h fhat_{reg P}(P) - sum_{Q on the box boundary} A_PQ gB(Q)
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
  const double* f = a.fhat ? a.fhat + (int64_t)a.region[i] * g.n_nodes : nullptr;
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
  a.F[i] = s;
}

struct RhsCorrArgs {
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

struct NdArgs {
  GridDesc g;
  int nC;
  int lin[3];
  int64_t n_dof;
  const int *d2s, *meta;
  const double *spos, *snrm, *U, *v, *Cg;
  const int8_t* region;
  double *dn_in, *dn_out, *Apsi;
};

// corrected tensor-product Lagrange interpolation of degree q = p on the
// (q+1)^d block centred at floor(t + 1/2), clamped into the grid (Sec. 5.5)
__global__ void k_normal_derivative(NdArgs a) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n_dof) return;
  const GridDesc& g = a.g;
  const int q = g.p;
  int s = a.d2s[c];
  int k = a.meta[(int64_t)s * 5 + 3];
  const double* P = a.spos + (int64_t)s * g.d;
  const double* nv = a.snrm + (int64_t)s * g.d;
  int st[3] = {0, 0, 0};
  double val[3][5], der[3][5];
  for (int ax = 0; ax < 3; ++ax)
    for (int j = 0; j < 5; ++j) val[ax][j] = (ax < g.d ? 0.0 : (j == 0 ? 1.0 : 0.0)), der[ax][j] = 0.0;
  for (int ax = 0; ax < g.d; ++ax) {
    double t = (P[ax] - g.lo) / g.h;
    int b0 = (int)floor(t + 0.5) - q / 2;
    if (b0 < 0) b0 = 0;
    if (b0 > g.N - q) b0 = g.N - q;
    st[ax] = b0;
    double u = t - (double)b0;
    for (int j = 0; j <= q; ++j) {
      double v = 1.0;
      for (int m = 0; m <= q; ++m)
        if (m != j) v = v * (u - (double)m) / (double)(j - m);
      val[ax][j] = v;
      double dv = 0.0;
      for (int l = 0; l <= q; ++l) {
        if (l == j) continue;
        double w = 1.0 / (double)(j - l);
        for (int m = 0; m <= q; ++m)
          if (m != j && m != l) w = w * (u - (double)m) / (double)(j - m);
        dv += w;
      }
      der[ax][j] = dv;
    }
  }
  double grad[3] = {0.0, 0.0, 0.0};
  int nz = g.d == 3 ? q + 1 : 1;
  for (int b2 = 0; b2 < nz; ++b2)
    for (int b1 = 0; b1 <= q; ++b1)
      for (int b0 = 0; b0 <= q; ++b0) {
        int64_t Q = ravel(g, st[0] + b0, st[1] + b1, st[2] + b2);
        int rq = a.region[Q];
        double vt = a.v[Q];
        if (rq != k) vt += Cval(a.Cg, g.n_nodes, k, Q) - Cval(a.Cg, g.n_nodes, rq, Q);
        int bb[3] = {b0, b1, b2};
        for (int ax = 0; ax < g.d; ++ax) {
          double w = der[ax][bb[ax]] / g.h;
          for (int b = 0; b < g.d; ++b)
            if (b != ax) w = w * val[b][bb[b]];
          grad[ax] += w * vt;
        }
      }
  double dn = 0.0, dnC = 0.0;
  const double* Uc = a.U + c * (int64_t)a.nC;
  for (int ax = 0; ax < g.d; ++ax) {
    dn += nv[ax] * grad[ax];
    dnC += nv[ax] * Uc[a.lin[ax]];
  }
  dnC = dnC / g.h;
  double dout = dn - dnC;
  if (a.dn_in) a.dn_in[c] = dn;
  if (a.dn_out) a.dn_out[c] = dout;
  if (a.Apsi) a.Apsi[c] = (g.beta_in * dn - g.beta_out * dout) / (g.beta_in + g.beta_out);
}

__global__ void k_bie_rhs(GridDesc g, int64_t n_dof, const int* d2s, const double* g2, const double* dn_in,
                          const double* dn_out, double* b) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_dof) return;
  double J = g.beta_in * dn_in[c] - g.beta_out * dn_out[c];
  b[c] = (g2[d2s[c]] - J) / (g.beta_in + g.beta_out);
}

}  // namespace

// ---------------------------------------------------------------- launchers
void op_extend(kfbi_plan* pl, const double* psi, double* psiS) {
  hipLaunchKernelGGL(k_extend, dim3(nb(pl->n_surf)), dim3(KFBI_BLOCK), 0, pl->stream, pl->n_surf, pl->g.p,
                     pl->ext_idx, pl->ext_w, psi, psiS);
}

void op_coefficients(kfbi_plan* pl, const double* a, const double* b, const double* ftilde) {
  CoefArgs A{pl->n_dof, pl->nC, pl->nP, pl->nD, pl->nN, pl->g.h, pl->MinvT, a, b, ftilde, pl->stD, pl->stN, pl->U};
  hipLaunchKernelGGL(k_coef, dim3(nb(pl->n_dof * pl->nC)), dim3(KFBI_BLOCK), 0, pl->stream, A);
}

void op_correction_values(kfbi_plan* pl) {
  if (pl->n_corr == 0) return;
  CorrArgs A{pl->g, make_mono(pl), pl->n_corr, pl->ce_k, pl->ce_node, pl->ce_owner, pl->d2s, pl->s_pos, pl->U,
             pl->Cg};
  hipLaunchKernelGGL(k_corr_values, dim3(nb(pl->n_corr)), dim3(KFBI_BLOCK), 0, pl->stream, A);
}

void op_rhs_base(kfbi_plan* pl, const double* fhat, const double* gB, double* F) {
  RhsArgs A{pl->g, make_stencil(pl->g), pl->region, fhat, gB, F};
  hipLaunchKernelGGL(k_rhs_base, dim3(nb(pl->g.n_nodes)), dim3(KFBI_BLOCK), 0, pl->stream, A);
}

void op_rhs_correct(kfbi_plan* pl, double* F, bool overwrite) {
  if (pl->n_irr == 0) return;
  RhsCorrArgs A{pl->g, make_stencil(pl->g), pl->n_irr, pl->irr, pl->region, pl->Cg, F, overwrite ? 1 : 0};
  hipLaunchKernelGGL(k_rhs_correct, dim3(nb(pl->n_irr)), dim3(KFBI_BLOCK), 0, pl->stream, A);
}

void op_boundary(kfbi_plan* pl, const double* gB, double* v) {
  hipLaunchKernelGGL(k_boundary, dim3(nb(pl->g.n_nodes)), dim3(KFBI_BLOCK), 0, pl->stream, pl->g, gB, v);
}

void op_normal_derivatives(kfbi_plan* pl, const double* v, double* dn_in, double* dn_out, double* Apsi) {
  NdArgs A;
  A.g = pl->g;
  A.nC = pl->nC;
  for (int ax = 0; ax < 3; ++ax) A.lin[ax] = ax + 1;   // graded order: 1, x, y(, z)
  A.n_dof = pl->n_dof;
  A.d2s = pl->d2s;
  A.meta = pl->s_meta;
  A.spos = pl->s_pos;
  A.snrm = pl->s_nrm;
  A.U = pl->U;
  A.v = v;
  A.Cg = pl->Cg;
  A.region = pl->region;
  A.dn_in = dn_in;
  A.dn_out = dn_out;
  A.Apsi = Apsi;
  hipLaunchKernelGGL(k_normal_derivative, dim3(nb(pl->n_dof)), dim3(KFBI_BLOCK), 0, pl->stream, A);
}

void op_bie_rhs(kfbi_plan* pl, const double* g2, const double* dn_in, const double* dn_out, double* b) {
  hipLaunchKernelGGL(k_bie_rhs, dim3(nb(pl->n_dof)), dim3(KFBI_BLOCK), 0, pl->stream, pl->g, pl->n_dof, pl->d2s,
                     g2, dn_in, dn_out, b);
}
