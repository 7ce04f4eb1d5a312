// Step S0 -- geometry of the simple interface problem on the device.
//
// Paper: Sec. 5.1 (level set, grid-line intersections by bisection, normals,
// overlapping surface sets Gamma_r = {|n_r| > cos alpha}, reference plane of
// the largest normal component), Sec. 5.2 (regular / irregular nodes),
// Sec. 5.3 (closest-primary-point partition of unity), Sec. 5.4 (collocation
// lattices), Sec. 5.5 (interpolation blocks).  Where the paper leaves a
// choice open, the rules below are the library's readings; every discrete
// decision is a function of IEEE-exact operations only (+ - * / sqrt floor,
// compiled without contraction), so it is reproducible on any IEEE machine.
//
// Surface points are kept in canonical order (family r, line id, segment,
// interface) by order-preserving stream compaction; no sort is needed.
#include <math.h>
#include <stdio.h>

#include <algorithm>
#include <array>
#include <cstdlib>
#include <vector>

#include "kfbi_internal.h"

#pragma clang fp contract(off)

namespace {

constexpr int CMP_IT = 4;     // items per thread of a compaction block (more blocks, shorter serial chains)
constexpr int CMP_CH = KFBI_BLOCK * CMP_IT;
constexpr int BISECT_STEPS = 52;
constexpr int MARGIN = 3;
constexpr double TIE_BAND = 1e-12;

struct LSet {
  int K;
  int kind[KFBI_MAX_IFACE];
  double p[KFBI_MAX_IFACE][KFBI_LS_NPARAM];
  // sampled level sets: the plan's copy of the node samples, and the grid
  const double* S[KFBI_MAX_IFACE];
  double lo, h;
  int N, d;
};

// Collocation lattices and window shifts (host-built, mirrors of the lattice
// rules documented in collocation.hip).
struct Lattices {
  int nD, nN, nSD, nSN;
  int offD[KFBI_MAXD][2];
  int offN[KFBI_MAXN][2];
  int shD[81][2];
  int shN[81][2];
};

// ---------------------------------------------------------------- level sets
// exp(t), t <= 0, with +, -, *, / only: the degree-12 Taylor polynomial of
// exp at t / 1024 in Horner form, squared ten times (relative error about
// 1e-13 on [-40, 0]); the molecular level set is defined with it, so its
// value at a point is an exact function of the inputs
__device__ double exp_arith(double t) {
  const double y = t / 1024.0;
  double s = 1.0;
  for (int k = 12; k >= 1; --k) s = 1.0 + y * s / (double)k;
  for (int i = 0; i < 10; ++i) s = s * s;
  return s;
}

// Sampled level set (the level set known only at the grid nodes): the
// tensor-product Lagrange interpolant of degree q on the (q+1)^d nodes
// around the point's cell, per axis base floor(t) - (q-1)/2 clamped to
// [0, N-q], t = (x - lo)/h snapped to the nearest integer within 1e-9 (on a
// grid line the interpolant is the line's 1D one, at a node the sample).
// grad != null: the gradient of the same polynomial instead of the value.
constexpr int LS_QMAX = 5;
__device__ double ls_grid(const LSet& L, int k, const double X[3], double* grad) {
  const int q = (int)L.p[k][0];
  int base[3] = {0, 0, 0};
  // value: an axis on which the point sits at a node has one nonzero
  // weight (exactly 1); the zero terms are skipped, which leaves the sum
  // bit for bit unchanged (they add +-0)
  int jlo[3] = {0, 0, 0}, jhi[3] = {q, q, q};
  double W[3][LS_QMAX + 1], D[3][LS_QMAX + 1];
  for (int a = 0; a < L.d; ++a) {
    double t = (X[a] - L.lo) / L.h;
    const double r = floor(t + 0.5);
    const bool snap = fabs(t - r) < 1e-9;
    if (snap) t = r;
    int b = (int)floor(t) - (q - 1) / 2;
    if (b < 0) b = 0;
    if (b > L.N - q) b = L.N - q;
    base[a] = b;
    if (snap && !grad) jlo[a] = jhi[a] = (int)t - b;
    const double u = t - (double)b;
    for (int j = 0; j <= q; ++j) {
      double v = 1.0;
      for (int m = 0; m <= q; ++m)
        if (m != j) v = v * (u - (double)m) / (double)(j - m);
      double dv = 0.0;
      for (int l = 0; l <= q; ++l) {
        if (l == j) continue;
        double w = 1.0 / (double)(j - l);
        for (int m = 0; m <= q; ++m)
          if (m != j && m != l) w = w * (u - (double)m) / (double)(j - m);
        dv = dv + w;
      }
      W[a][j] = v;
      D[a][j] = dv;
    }
  }
  const double* S = L.S[k];
  const int64_t n1 = L.N + 1;
  if (L.d == 2) jlo[2] = jhi[2] = 0;
  double val = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
  for (int j2 = jlo[2]; j2 <= jhi[2]; ++j2)
    for (int j1 = jlo[1]; j1 <= jhi[1]; ++j1)
      for (int j0 = jlo[0]; j0 <= jhi[0]; ++j0) {
        int64_t idx = (int64_t)(base[0] + j0) + (int64_t)(base[1] + j1) * n1;
        if (L.d == 3) idx = idx + (int64_t)(base[2] + j2) * (n1 * n1);
        const double s = S[idx];
        if (!grad) {
          double w = W[0][j0] * W[1][j1];
          if (L.d == 3) w = w * W[2][j2];
          val = val + w * s;
        } else {
          double c0 = D[0][j0] * W[1][j1], c1 = W[0][j0] * D[1][j1];
          if (L.d == 3) {
            c0 = c0 * W[2][j2];
            c1 = c1 * W[2][j2];
            g2 = g2 + (W[0][j0] * W[1][j1] * D[2][j2]) * s;
          }
          g0 = g0 + c0 * s;
          g1 = g1 + c1 * s;
        }
      }
  if (grad) {
    grad[0] = g0 / L.h;
    grad[1] = g1 / L.h;
    grad[2] = L.d == 3 ? g2 / L.h : 0.0;
  }
  return val;
}

__device__ double ls_value(const LSet& L, int k, double x, double y, double z) {
  const double* p = L.p[k];
  switch (L.kind[k]) {
    case KFBI_LS_GRID: {
      const double X[3] = {x, y, z};
      return ls_grid(L, k, X, nullptr);
    }
    case KFBI_LS_ELLIPSE2D: {
      double dx = x - p[0], dy = y - p[1];
      double XX = p[2] * dx + p[3] * dy;
      double YY = p[2] * dy - p[3] * dx;
      double Xa = XX / p[4], Yb = YY / p[5];
      return Xa * Xa + Yb * Yb - 1.0;
    }
    case KFBI_LS_STAR2D: {
      double dx = x - p[0], dy = y - p[1];
      double rho = sqrt(dx * dx + dy * dy);
      if (rho == 0.0) return -p[2];
      double ux = dx / rho, uy = dy / rho;
      double cr = 1.0, ci = 0.0, r = 0.0 + p[2];
      for (int k = 1; k <= 8; ++k) {
        double ncr = cr * ux - ci * uy;
        double nci = cr * uy + ci * ux;
        cr = ncr;
        ci = nci;
        r = r + (p[2 + k] * cr + p[10 + k] * ci);
      }
      return rho - r;
    }
    case KFBI_LS_SPHERE3D: {
      double d0 = x - p[0], d1 = y - p[1], d2 = z - p[2];
      return d0 * d0 + d1 * d1 + d2 * d2 - p[3] * p[3];
    }
    case KFBI_LS_ELLIPSOID3D: {
      double d0 = x - p[0], d1 = y - p[1], d2 = z - p[2];
      const double* R = p + 6;
      double s = 0.0;
      double Xa0, Xa1, Xa2;
      {
        double X0 = R[0] * d0 + R[3] * d1 + R[6] * d2;
        double X1 = R[1] * d0 + R[4] * d1 + R[7] * d2;
        double X2 = R[2] * d0 + R[5] * d1 + R[8] * d2;
        Xa0 = X0 / p[3];
        Xa1 = X1 / p[4];
        Xa2 = X2 / p[5];
      }
      s = Xa0 * Xa0 + Xa1 * Xa1 + Xa2 * Xa2 - 1.0;
      return s;
    }
    case KFBI_LS_TORUS3D: {
      double d0 = x - p[0], d1 = y - p[1], d2 = z - p[2];
      double rho = sqrt(d0 * d0 + d1 * d1);
      double q = rho - p[3];
      return q * q + d2 * d2 - p[4] * p[4];
    }
    case KFBI_LS_PRODUCT3D: {
      double X = p[3] * (x - p[0]), Y = p[3] * (y - p[1]), Z = p[3] * (z - p[2]);
      double x2 = X * X, y2 = Y * Y, z2 = Z * Z;
      return (1.0 + x2) * (1.0 + y2) * (1.0 + z2) + 8.0 * X * Y * Z + x2 + y2 + z2 - 3.0;
    }
    case KFBI_LS_MOLECULE3D: {
      const double rr = p[1] * p[1];
      const int m = (int)p[2];
      double H = p[0];
      for (int a = 0; a < m; ++a) {
        double d0 = x - p[3 + 3 * a], d1 = y - p[4 + 3 * a], d2 = z - p[5 + 3 * a];
        H = H - exp_arith(-(d0 * d0 + d1 * d1 + d2 * d2) / rr);
      }
      return H;
    }
  }
  return 1.0;
}

__device__ void ls_grad(const LSet& L, int k, double x, double y, double z, double g[3]) {
  const double* p = L.p[k];
  g[0] = g[1] = g[2] = 0.0;
  switch (L.kind[k]) {
    case KFBI_LS_GRID: {
      const double X[3] = {x, y, z};
      (void)ls_grid(L, k, X, g);
      return;
    }
    case KFBI_LS_ELLIPSE2D: {
      double dx = x - p[0], dy = y - p[1];
      double XX = p[2] * dx + p[3] * dy;
      double YY = p[2] * dy - p[3] * dx;
      double Xa = XX / p[4], Yb = YY / p[5];
      double GX = 2.0 * Xa / p[4], GY = 2.0 * Yb / p[5];
      g[0] = GX * p[2] - GY * p[3];
      g[1] = GX * p[3] + GY * p[2];
      return;
    }
    case KFBI_LS_STAR2D: {
      double dx = x - p[0], dy = y - p[1];
      double rho = sqrt(dx * dx + dy * dy);
      double safe = rho == 0.0 ? 1.0 : rho;
      double ux = dx / safe, uy = dy / safe;
      double cr = 1.0, ci = 0.0, rp = 0.0;
      for (int k = 1; k <= 8; ++k) {
        double ncr = cr * ux - ci * uy;
        double nci = cr * uy + ci * ux;
        cr = ncr;
        ci = nci;
        rp = rp + (double)k * (p[10 + k] * cr - p[2 + k] * ci);
      }
      g[0] = ux + rp * uy / safe;
      g[1] = uy - rp * ux / safe;
      return;
    }
    case KFBI_LS_SPHERE3D:
      g[0] = 2.0 * (x - p[0]);
      g[1] = 2.0 * (y - p[1]);
      g[2] = 2.0 * (z - p[2]);
      return;
    case KFBI_LS_ELLIPSOID3D: {
      double d0 = x - p[0], d1 = y - p[1], d2 = z - p[2];
      const double* R = p + 6;
      double X0 = R[0] * d0 + R[3] * d1 + R[6] * d2;
      double X1 = R[1] * d0 + R[4] * d1 + R[7] * d2;
      double X2 = R[2] * d0 + R[5] * d1 + R[8] * d2;
      double G0 = 2.0 * (X0 / p[3]) / p[3];
      double G1 = 2.0 * (X1 / p[4]) / p[4];
      double G2 = 2.0 * (X2 / p[5]) / p[5];
      for (int i = 0; i < 3; ++i) g[i] = R[i * 3 + 0] * G0 + R[i * 3 + 1] * G1 + R[i * 3 + 2] * G2;
      return;
    }
    case KFBI_LS_TORUS3D: {
      double d0 = x - p[0], d1 = y - p[1], d2 = z - p[2];
      double rho = sqrt(d0 * d0 + d1 * d1);
      double q = rho - p[3];
      double safe = rho == 0.0 ? 1.0 : rho;
      g[0] = 2.0 * q * d0 / safe;
      g[1] = 2.0 * q * d1 / safe;
      g[2] = 2.0 * d2;
      return;
    }
    case KFBI_LS_PRODUCT3D: {
      double X = p[3] * (x - p[0]), Y = p[3] * (y - p[1]), Z = p[3] * (z - p[2]);
      double x2 = X * X, y2 = Y * Y, z2 = Z * Z;
      double gx = 2.0 * X * (1.0 + y2) * (1.0 + z2) + 8.0 * Y * Z + 2.0 * X;
      double gy = 2.0 * Y * (1.0 + x2) * (1.0 + z2) + 8.0 * X * Z + 2.0 * Y;
      double gz = 2.0 * Z * (1.0 + x2) * (1.0 + y2) + 8.0 * X * Y + 2.0 * Z;
      g[0] = p[3] * gx;
      g[1] = p[3] * gy;
      g[2] = p[3] * gz;
      return;
    }
    case KFBI_LS_MOLECULE3D: {
      const double rr = p[1] * p[1];
      const int m = (int)p[2];
      for (int a = 0; a < m; ++a) {
        double d0 = x - p[3 + 3 * a], d1 = y - p[4 + 3 * a], d2 = z - p[5 + 3 * a];
        double e = exp_arith(-(d0 * d0 + d1 * d1 + d2 * d2) / rr);
        g[0] = g[0] + 2.0 * e * d0 / rr;
        g[1] = g[1] + 2.0 * e * d1 / rr;
        g[2] = g[2] + 2.0 * e * d2 / rr;
      }
      return;
    }
  }
}

__device__ __forceinline__ double node_x(const GridDesc& g, int i) { return g.lo + (double)i * g.h; }

// node indices fit 32 bits ((N+1)^3 < 2^31 for N <= 1024)
__device__ __forceinline__ void unravel(const GridDesc& g, int64_t idx, int c[3]) {
  const unsigned u = (unsigned)idx, n1 = (unsigned)g.n1;
  const unsigned r = u / n1;
  c[0] = (int)(u - r * n1);
  c[1] = (int)(r % n1);
  c[2] = g.d == 2 ? 0 : (int)(r / n1);
}

__device__ __forceinline__ int64_t ravel(const GridDesc& g, const int c[3]) {
  return (int64_t)c[0] + (int64_t)g.n1 * ((int64_t)c[1] + (g.d == 3 ? (int64_t)g.n1 * c[2] : 0));
}

__device__ __forceinline__ void trans_axes(int d, int r, int T[2]) {
  int j = 0;
  for (int a = 0; a < d; ++a)
    if (a != r) T[j++] = a;
}

// line id of the family-r line through the integer coordinates c[b], b != r
__device__ __forceinline__ int64_t line_id(const GridDesc& g, int r, const int c[3]) {
  int T[2];
  trans_axes(g.d, r, T);
  int64_t lid = c[T[0]];
  if (g.d == 3) lid += (int64_t)g.n1 * c[T[1]];
  return lid;
}

// ---------------------------------------------------------------- compaction
__device__ __forceinline__ int wave_sum(int v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

template <class Pred>
__global__ void __launch_bounds__(KFBI_BLOCK) k_count(int64_t n, Pred pred, int* blk) {
  int64_t base = (int64_t)blockIdx.x * CMP_CH;
  int c = 0;
  for (int j = 0; j < CMP_IT; ++j) {
    int64_t i = base + (int64_t)j * KFBI_BLOCK + threadIdx.x;
    if (i < n && pred(i)) ++c;
  }
  __shared__ int red[KFBI_BLOCK / 64];
  c = wave_sum(c);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int w = 0; w < KFBI_BLOCK / 64; ++w) s += red[w];
    blk[blockIdx.x] = s;
  }
}

// as k_count, also storing the predicate per item (later compaction passes
// read the flag instead of re-evaluating the predicate)
template <class Pred>
__global__ void __launch_bounds__(KFBI_BLOCK) k_count_flags(int64_t n, Pred pred, int* blk, uint8_t* flags) {
  int64_t base = (int64_t)blockIdx.x * CMP_CH;
  int c = 0;
  for (int j = 0; j < CMP_IT; ++j) {
    int64_t i = base + (int64_t)j * KFBI_BLOCK + threadIdx.x;
    if (i < n) {
      bool f = pred(i);
      flags[i] = f ? 1 : 0;
      c += f ? 1 : 0;
    }
  }
  __shared__ int red[KFBI_BLOCK / 64];
  c = wave_sum(c);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int w = 0; w < KFBI_BLOCK / 64; ++w) s += red[w];
    blk[blockIdx.x] = s;
  }
}

// exclusive scan of blk[0..nb) in place (one block of 1024 threads, each
// owning a contiguous chunk; wave-level shuffle scans, two barriers);
// total -> *tot
__global__ void __launch_bounds__(1024) k_scan(int* blk, int64_t nb, int* tot) {
  __shared__ long long wpre[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t per = (nb + 1023) / 1024;
  int64_t b0 = (int64_t)threadIdx.x * per;
  int64_t b1 = b0 + per < nb ? b0 + per : nb;
  long long s = 0;
  for (int64_t i = b0; i < b1; ++i) s += blk[i];
  long long v = s;
  for (int off = 1; off < 64; off <<= 1) {
    long long n = __shfl_up(v, off, 64);
    if (lane >= off) v += n;
  }
  if (lane == 63) wpre[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long run = 0;
    for (int w = 0; w < 16; ++w) {
      long long t = wpre[w];
      wpre[w] = run;
      run += t;
    }
    *tot = (int)run;
  }
  __syncthreads();
  long long run = wpre[wave] + v - s;
  for (int64_t i = b0; i < b1; ++i) {
    int t = blk[i];
    blk[i] = (int)run;
    run += t;
  }
}

// device-wide exclusive scan out[i] = sum_{j<i} in[j]: block sums, scan of
// the block sums, then a block-local scan per chunk (coalesced, in order)
__global__ void __launch_bounds__(KFBI_BLOCK) k_scan_sums(int64_t n, const int* in, int* blk) {
  int64_t base = (int64_t)blockIdx.x * CMP_CH;
  int c = 0;
  for (int j = 0; j < CMP_IT; ++j) {
    int64_t i = base + (int64_t)j * KFBI_BLOCK + threadIdx.x;
    if (i < n) c += in[i];
  }
  __shared__ int red[KFBI_BLOCK / 64];
  c = wave_sum(c);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int w = 0; w < KFBI_BLOCK / 64; ++w) s += red[w];
    blk[blockIdx.x] = s;
  }
}

__global__ void __launch_bounds__(KFBI_BLOCK) k_scan_apply(int64_t n, const int* in, int* out, const int* blk) {
  __shared__ int wtot[KFBI_BLOCK / 64];
  int64_t base = (int64_t)blockIdx.x * CMP_CH;
  int run = blk[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = 0; j < CMP_IT; ++j) {
    int64_t i = base + (int64_t)j * KFBI_BLOCK + threadIdx.x;
    int x = i < n ? in[i] : 0;
    int v = x;
    for (int off = 1; off < 64; off <<= 1) {
      int y = __shfl_up(v, off, 64);
      if (lane >= off) v += y;
    }
    if (lane == 63) wtot[wave] = v;
    __syncthreads();
    int pre = 0, tot = 0;
    for (int w = 0; w < KFBI_BLOCK / 64; ++w) {
      if (w < wave) pre += wtot[w];
      tot += wtot[w];
    }
    if (i < n) out[i] = run + pre + v - x;
    run += tot;
    __syncthreads();
  }
}

template <class Pred, class Emit>
__global__ void __launch_bounds__(KFBI_BLOCK) k_emit(int64_t n, Pred pred, Emit emit, const int* blk) {
  __shared__ int wtot[KFBI_BLOCK / 64];
  int64_t base = (int64_t)blockIdx.x * CMP_CH;
  int run = blk[blockIdx.x];
  int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = 0; j < CMP_IT; ++j) {
    int64_t i = base + (int64_t)j * KFBI_BLOCK + threadIdx.x;
    bool f = i < n && pred(i);
    unsigned long long m = __ballot(f);
    int r = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wtot[wave] = __popcll(m);
    __syncthreads();
    int pre = 0, tot = 0;
    for (int w = 0; w < KFBI_BLOCK / 64; ++w) {
      if (w < wave) pre += wtot[w];
      tot += wtot[w];
    }
    if (f) emit(i, run + pre + r);
    run += tot;
    __syncthreads();
  }
}

// ---------------------------------------------------------------- predicates / emitters
struct RegionArgs {
  GridDesc g;
  LSet L;
  int8_t* region;
  int* flags;
};

__global__ void k_regions(RegionArgs a) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.g.n_nodes) return;
  int c[3];
  unravel(a.g, i, c);
  double x = node_x(a.g, c[0]), y = node_x(a.g, c[1]), z = a.g.d == 3 ? node_x(a.g, c[2]) : 0.0;
  int reg = 0, fl = 0;
  for (int k = 0; k < a.L.K; ++k) {
    // a sampled level set at a node is its sample (the interpolant's
    // weights there are exactly one and zeros)
    const double hv = a.L.kind[k] == KFBI_LS_GRID ? a.L.S[k][i] : ls_value(a.L, k, x, y, z);
    if (hv < 0.0) {
      if (reg != 0) fl |= FLAG_OVERLAP;
      reg = k + 1;
    }
  }
  if (reg != 0) {
    for (int ax = 0; ax < a.g.d; ++ax)
      if (c[ax] < MARGIN || c[ax] > a.g.N - MARGIN) fl |= FLAG_MARGIN;
  }
  a.region[i] = (int8_t)reg;
  if (fl) atomicOr(a.flags, fl);
}

struct SegInfo {
  int r, s;
  int64_t lid, a, b;
};

__device__ __forceinline__ SegInfo seg_info(const GridDesc& g, int64_t seg) {
  SegInfo o;
  const unsigned L = g.d == 2 ? (unsigned)g.n1 : (unsigned)g.n1 * (unsigned)g.n1;
  const int logN = __ffs(g.N) - 1;                 // N is a power of two
  o.s = (int)(seg & (g.N - 1));
  const unsigned rest = (unsigned)(seg >> logN);   // < d (N+1)^(d-1)
  const unsigned r = rest / L;
  o.r = (int)r;
  const unsigned lid = rest - r * L;
  o.lid = lid;
  int T[2];
  trans_axes(g.d, o.r, T);
  int c[3] = {0, 0, 0};
  const unsigned l1 = lid / (unsigned)g.n1;
  c[T[0]] = (int)(lid - l1 * (unsigned)g.n1);
  if (g.d == 3) c[T[1]] = (int)l1;
  c[o.r] = o.s;
  o.a = ravel(g, c);
  c[o.r] = o.s + 1;
  o.b = ravel(g, c);
  return o;
}

__device__ __forceinline__ int64_t item_seg(const GridDesc& g, int64_t item, int* k) {
  if (g.K == 1) {
    *k = 1;
    return item;
  }
  int64_t seg = item / g.K;
  *k = (int)(item - seg * g.K) + 1;
  return seg;
}

struct CandPred {
  GridDesc g;
  const int8_t* region;
  __device__ bool operator()(int64_t item) const {
    int k;
    int64_t seg = item_seg(g, item, &k);
    SegInfo si = seg_info(g, seg);
    return (region[si.a] == k) != (region[si.b] == k);
  }
};

struct CandEmit {
  GridDesc g;
  const int8_t* region;
  int *r, *lid, *segs, *k, *ina;
  __device__ void operator()(int64_t item, int pos) const {
    int kk;
    int64_t seg = item_seg(g, item, &kk);
    SegInfo si = seg_info(g, seg);
    r[pos] = si.r;
    lid[pos] = (int)si.lid;
    segs[pos] = si.s;
    k[pos] = kk;
    ina[pos] = region[si.a] == kk;
  }
};

struct BisectArgs {
  GridDesc g;
  LSet L;
  int64_t n;
  const int *r, *lid, *seg, *k, *ina;
  double *pos, *nrm;
  int* acc;
};

// Bisection of BISECT_STEPS halvings, six halvings per round: one
// wavefront per candidate, lane L evaluates the midpoint of heap node L of
// the next six levels (63 nodes), found by halving along the node's path
// from the current endpoints, and the sequential decisions are replayed on
// the wavefront's ballot.  Every midpoint is 0.5*(lo+hi) of the same
// endpoints as in plain bisection, so the root is identical; 9 rounds
// instead of 52 sequential evaluations.
constexpr int BIS_G = 64;
constexpr int BIS_LEV = 6;
__global__ void __launch_bounds__(KFBI_BLOCK) k_bisect(BisectArgs a) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t i = t / BIS_G;
  int lane = (int)(t % BIS_G);
  if (i >= a.n) return;               // whole wavefronts leave together
  const GridDesc& g = a.g;
  int r = a.r[i], k = a.k[i] - 1;
  int T[2];
  trans_axes(g.d, r, T);
  double X[3] = {0.0, 0.0, 0.0};
  int lid = a.lid[i];
  X[T[0]] = node_x(g, lid % g.n1);
  if (g.d == 3) X[T[1]] = node_x(g, lid / g.n1);
  double xr0 = g.lo + (double)a.seg[i] * g.h;
  bool ina = a.ina[i] != 0;
  double tlo = 0.0, thi = 1.0;
  int left = BISECT_STEPS;
  // heap node of this lane: level lv, path bits of lane + 1 below its leading one
  const unsigned hl = (unsigned)lane + 1u;
  const int lv = 31 - __clz((int)hl);
  while (left > 0) {
    const int depth = left >= BIS_LEV ? BIS_LEV : left;
    bool mine = false;
    if (lv < depth) {
      double lo = tlo, hi = thi;
      for (int b = lv - 1; b >= 0; --b) {
        const double mid = 0.5 * (lo + hi);
        if ((hl >> b) & 1u)
          lo = mid;
        else
          hi = mid;
      }
      X[r] = xr0 + 0.5 * (lo + hi) * g.h;
      mine = ls_value(a.L, k, X[0], X[1], X[2]) < 0.0;
    }
    const unsigned long long bits = __ballot(mine);
    int node = 0;   // heap index of the midpoint used at this level
    for (int lev = 0; lev < depth; ++lev) {
      const double mid = 0.5 * (tlo + thi);
      const bool inside = (bits >> node) & 1ull;
      const bool right = inside == ina;     // same side as the start: root is to the right
      if (right)
        tlo = mid;
      else
        thi = mid;
      node = 2 * node + (right ? 2 : 1);
    }
    left -= depth;
  }
  if (lane != 0) return;
  double tr = 0.5 * (tlo + thi);
  X[r] = xr0 + tr * g.h;
  double G[3];
  ls_grad(a.L, k, X[0], X[1], X[2], G);
  double s = G[0] * G[0] + G[1] * G[1];
  if (g.d == 3) s = s + G[2] * G[2];
  double nr = sqrt(s);
  double n[3] = {G[0] / nr, G[1] / nr, g.d == 3 ? G[2] / nr : 0.0};
  for (int ax = 0; ax < g.d; ++ax) {
    a.pos[i * g.d + ax] = X[ax];
    a.nrm[i * g.d + ax] = n[ax];
  }
  a.acc[i] = fabs(n[r]) > g.cos_alpha;
}

struct AccPred {
  const int* acc;
  __device__ bool operator()(int64_t i) const { return acc[i] != 0; }
};

struct SurfEmit {
  int d;
  const double *cpos, *cnrm;
  const int *r, *lid, *seg, *k;
  double *pos, *nrm;
  int* meta;
  __device__ void operator()(int64_t i, int o) const {
    double best = -1.0;
    int arg = 0;
    for (int ax = 0; ax < d; ++ax) {
      pos[(int64_t)o * d + ax] = cpos[i * d + ax];
      nrm[(int64_t)o * d + ax] = cnrm[i * d + ax];
      double v = fabs(cnrm[i * d + ax]);
      if (ax == 0 || v > best) {
        best = v;
        arg = ax;
      }
    }
    meta[(int64_t)o * 5 + 0] = r[i];
    meta[(int64_t)o * 5 + 1] = lid[i];
    meta[(int64_t)o * 5 + 2] = seg[i];
    meta[(int64_t)o * 5 + 3] = k[i];
    meta[(int64_t)o * 5 + 4] = arg == r[i];
  }
};

// line CSR of the surface table; also resets the surface-to-DOF map (-1)
// and the stencil-use flags of every surface point
__global__ void k_lines(int64_t n, int64_t L, const int* meta, int* ls, int* le, int* s2d, uint8_t* s_need) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  s2d[i] = -1;
  s_need[i] = 0;
  int64_t key = (int64_t)meta[i * 5] * L + meta[i * 5 + 1];
  int64_t kp = i > 0 ? (int64_t)meta[(i - 1) * 5] * L + meta[(i - 1) * 5 + 1] : -1;
  int64_t kn = i + 1 < n ? (int64_t)meta[(i + 1) * 5] * L + meta[(i + 1) * 5 + 1] : -1;
  if (kp != key) ls[key] = (int)i;
  if (kn != key) le[key] = (int)(i + 1);
}

struct PrimPred {
  const int* meta;
  __device__ bool operator()(int64_t i) const { return meta[i * 5 + 4] != 0; }
};

// the primary test of SurfEmit (family r equals the first axis of largest
// |normal component|) on an accepted candidate, before the surface table
// exists
__device__ __forceinline__ bool cand_primary(int d, const double* cnrm, const int* r, int64_t i) {
  double best = -1.0;
  int arg = 0;
  for (int ax = 0; ax < d; ++ax) {
    const double v = fabs(cnrm[i * d + ax]);
    if (ax == 0 || v > best) {
      best = v;
      arg = ax;
    }
  }
  return arg == r[i];
}

struct PrimCandPred {
  int d;
  const int *acc, *r;
  const double* cnrm;
  __device__ bool operator()(int64_t i) const { return acc[i] != 0 && cand_primary(d, cnrm, r, i); }
};

struct PrimEmit {
  int *d2s, *s2d;
  __device__ void operator()(int64_t i, int o) const {
    d2s[o] = (int)i;
    s2d[i] = o;
  }
};

// ---------------------------------------------------------------- stencils
struct SurfView {
  GridDesc g;
  const double *pos, *nrm;
  const int* meta;
  const int *ls, *le;
  int64_t L;
  __device__ int fam(int i) const { return meta[(int64_t)i * 5]; }
  __device__ int iface(int i) const { return meta[(int64_t)i * 5 + 3]; }
  __device__ bool prim(int i) const { return meta[(int64_t)i * 5 + 4] != 0; }
  __device__ double x(int i, int ax) const { return pos[(int64_t)i * g.d + ax]; }
  // nearest point of the interface of `ref` on line (r, lid) to xref along
  // e_r; primaries only if only_prim; -1 if none (distance in *bd)
  __device__ int nearest(int r, int64_t lid, int kref, double xref, bool only_prim, double* bd) const {
    int64_t key = (int64_t)r * L + lid;
    int bj = -1;
    double best = 0.0;
    for (int j = ls[key]; j < le[key]; ++j) {
      if (iface(j) != kref) continue;
      if (only_prim && !prim(j)) continue;
      double dd = fabs(x(j, r) - xref);
      if (bj < 0 || dd < best) {
        bj = j;
        best = dd;
      }
    }
    *bd = best;
    return bj;
  }
};

// the point of one window offset (o + s): the surface point of the centre's
// interface on the family-r line a0 + o + s nearest to the centre along e_r,
// or -1 if there is none, it fails the gate, or (need_prim) it is not primary
__device__ int pick_one(const SurfView& S, int i, int r, const int a0[2], const int o[2], const int s[2],
                        bool need_prim) {
  const GridDesc& g = S.g;
  int T[2];
  trans_axes(g.d, r, T);
  int c[3] = {0, 0, 0};
  int l1 = 0;
  for (int j = 0; j < g.d - 1; ++j) {
    int v = a0[j] + o[j] + s[j];
    if (v < 0 || v > g.N) return -1;
    c[T[j]] = v;
    int oo = o[j] + s[j];
    l1 += oo < 0 ? -oo : oo;
  }
  double bd;
  int bj = S.nearest(r, line_id(g, r, c), S.iface(i), S.x(i, r), false, &bd);
  if (bj < 0 || !(bd <= 2.0 * g.h * ((double)l1 + 1.0))) return -1;
  if (need_prim && !S.prim(bj)) return -1;
  return bj;
}

struct StencilArgs {
  SurfView S;
  Lattices lat;
  int64_t n_dof;
  const int* d2s;
  int *stD, *stN;
  uint8_t* s_need;
  int* flags;
};

constexpr int STG = 16;   // lanes per centre (>= the largest lattice, 15)

__device__ __forceinline__ bool group_all(bool v) {
  int x = v ? 1 : 0;
  for (int off = STG / 2; off > 0; off >>= 1) x &= __shfl_xor(x, off, STG);
  return x != 0;
}

// Collocation stencils, one group of STG lanes per centre: every window
// shift is tested with one lane per lattice offset (both lattices at once
// for a common shift), the first shift whose points are all valid wins
// (same order as a sequential search).  First one shift for both windows,
// from the Neumann lattice's list (its shifts keep offset 0 in both), with
// primary Neumann points only in a first pass when the Neumann data is a
// density (all kinds but the interior Dirichlet problem); failing that,
// each lattice on its own list.
__global__ void __launch_bounds__(KFBI_BLOCK) k_stencils(StencilArgs a) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t c = t / STG;
  int lane = (int)(t % STG);
  if (c >= a.n_dof) return;
  const SurfView& S = a.S;
  const GridDesc& g = S.g;
  int i = a.d2s[c];
  int r = S.fam(i);
  int T[2];
  trans_axes(g.d, r, T);
  int a0[2] = {0, 0};
  for (int j = 0; j < g.d - 1; ++j) a0[j] = (int)floor((S.x(i, T[j]) - g.lo) / g.h + 0.5);
  const int pass0 = g.bie == KFBI_BIE_DIRICHLET ? 1 : 0;   // 0: primary Neumann points first
  int pD = -1, pN = -1;
  bool okD = false, okN = false;
  for (int pass = pass0; pass < 2 && !okD; ++pass)
    for (int si = 0; si < a.lat.nSN && !okD; ++si) {
      int myD = lane < a.lat.nD ? pick_one(S, i, r, a0, a.lat.offD[lane], a.lat.shN[si], false) : 0;
      int myN = lane < a.lat.nN ? pick_one(S, i, r, a0, a.lat.offN[lane], a.lat.shN[si], pass == 0) : 0;
      if (group_all(myD >= 0 && myN >= 0)) {
        okD = okN = true;
        pD = myD;
        pN = myN;
      }
    }
  for (int si = 0; si < a.lat.nSD && !okD; ++si) {
    int my = lane < a.lat.nD ? pick_one(S, i, r, a0, a.lat.offD[lane], a.lat.shD[si], false) : 0;
    if (group_all(my >= 0)) {
      okD = true;
      pD = my;
    }
  }
  for (int pass = pass0; pass < 2 && !okN; ++pass)
    for (int si = 0; si < a.lat.nSN && !okN; ++si) {
      int my = lane < a.lat.nN ? pick_one(S, i, r, a0, a.lat.offN[lane], a.lat.shN[si], pass == 0) : 0;
      if (group_all(my >= 0)) {
        okN = true;
        pN = my;
      }
    }
  if (!okD || !okN) {
    if (lane == 0) atomicOr(a.flags, FLAG_UNRESOLVED_STENCIL);
    if (lane < a.lat.nD) a.stD[c * a.lat.nD + lane] = i;
    if (lane < a.lat.nN) a.stN[c * a.lat.nN + lane] = i;
    return;
  }
  if (lane < a.lat.nD) {
    a.stD[c * a.lat.nD + lane] = pD;
    // a density that is the jump [u] (Dirichlet problems, the two-density
    // form) is read by the collocation at the Dirichlet points
    if (S.g.bie == KFBI_BIE_DIRICHLET || S.g.bie == KFBI_BIE_TWO_DENSITY) a.s_need[pD] = 1;
  }
  if (lane < a.lat.nN) {
    a.stN[c * a.lat.nN + lane] = pN;
    a.s_need[pN] = 1;
  }
}

// ---------------------------------------------------------------- density extension
__device__ void lagrange(double u, const double* nodes, int n, double* w) {
  for (int j = 0; j < n; ++j) {
    double wj = 1.0;
    for (int m = 0; m < n; ++m)
      if (m != j) wj = wj * (u - nodes[m]) / (nodes[j] - nodes[m]);
    w[j] = wj;
  }
}

struct ExtArgs {
  SurfView S;
  int64_t n_surf;
  const int* s2d;
  const uint8_t* s_need;
  int* idx;
  double* w;
  int* flags;
};

// point of family F on the line through `coords` moved by o along `axis`,
// primary, of the interface of q, nearest to q along e_F; gate relative to oref
__device__ int ext_point(const SurfView& S, int q, int F, const int coords[3], int axis, int o,
                         int oref) {
  const GridDesc& g = S.g;
  int c[3] = {coords[0], coords[1], coords[2]};
  c[axis] = c[axis] + o;
  if (c[axis] < 0 || c[axis] > g.N) return -1;
  double bd;
  int bj = S.nearest(F, line_id(g, F, c), S.iface(q), S.x(q, F), true, &bd);
  int dof = o - oref;
  dof = dof < 0 ? -dof : dof;
  if (bj < 0 || !(bd <= 2.0 * g.h * ((double)dof + 1.0))) return -1;
  return bj;
}

constexpr int EXG = 8;    // lanes per surface point

// Density extension, one group of EXG lanes per surface point: lanes 0..4
// build the candidates (i) of the five shifts, lanes 0..7 test the eight
// own-family offsets of (ii); lane 0 then compares the candidates in the
// fixed order (i) shifts 0, 1, -1, 2, -2, then (ii) per transverse axis,
// and keeps the first with the smallest sum |w|.
__global__ void __launch_bounds__(KFBI_BLOCK) k_extension(ExtArgs a) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t q = t / EXG;
  int lane = (int)(t % EXG);
  if (q >= a.n_surf) return;
  const SurfView& S = a.S;
  const GridDesc& g = S.g;
  const int p = g.p;
  int* oi = a.idx + q * p;
  double* ow = a.w + q * p;
  if (S.prim((int)q)) {
    if (lane < p) {
      oi[lane] = lane == 0 ? a.s2d[q] : -1;
      ow[lane] = lane == 0 ? 1.0 : 0.0;
    }
    return;
  }
  if (!a.s_need[q]) {
    if (lane < p) {
      oi[lane] = -1;
      ow[lane] = 0.0;
    }
    return;
  }
  int r = S.fam((int)q);
  int rp = 0;
  double best = fabs(S.nrm[q * g.d]);
  for (int ax = 1; ax < g.d; ++ax) {
    double v = fabs(S.nrm[q * g.d + ax]);
    if (v > best) {
      best = v;
      rp = ax;
    }
  }
  int grid[3] = {0, 0, 0};
  for (int b = 0; b < g.d; ++b)
    if (b != r) grid[b] = (int)floor((S.x((int)q, b) - g.lo) / g.h + 0.5);
  double tq = (S.x((int)q, r) - g.lo) / g.h;
  int ft = (int)floor(tq);
  int base = ft - (p / 2 - 1);
  const int shifts[5] = {0, 1, -1, 2, -2};
  const int own[8] = {-1, 1, -2, 2, -3, 3, -4, 4};
  // (i) this lane's shift candidate
  bool cval = false;
  double cL = 0.0;
  int csel[4] = {0, 0, 0, 0};
  double cw[4] = {0.0, 0.0, 0.0, 0.0};
  if (lane < 5) {
    int c[3] = {grid[0], grid[1], grid[2]};
    c[r] = 0;
    double nodes[4];
    cval = true;
    for (int j = 0; j < p && cval; ++j) {
      int o = base + shifts[lane] + j;
      csel[j] = ext_point(S, (int)q, rp, c, r, o, ft);
      nodes[j] = (double)o;
      cval = csel[j] >= 0;
    }
    if (cval) {
      lagrange(tq, nodes, p, cw);
      for (int j = 0; j < p; ++j) cL = cL + fabs(cw[j]);
    }
  }
  bool have = false;
  double bestL = 0.0;
  int bsel[4] = {0, 0, 0, 0};
  double bw[4] = {0.0, 0.0, 0.0, 0.0};
  for (int si = 0; si < 5; ++si) {
    bool v = __shfl(cval ? 1 : 0, si, EXG) != 0;
    double L = __shfl(cL, si, EXG);
    int sl[4];
    double wl[4];
    for (int j = 0; j < 4; ++j) {
      sl[j] = __shfl(csel[j], si, EXG);
      wl[j] = __shfl(cw[j], si, EXG);
    }
    if (v && (!have || L < bestL)) {
      have = true;
      bestL = L;
      for (int j = 0; j < 4; ++j) {
        bsel[j] = sl[j];
        bw[j] = wl[j];
      }
    }
  }
  // (ii) own-family lines moved along each transverse axis
  int T[2];
  trans_axes(g.d, r, T);
  for (int tb = 0; tb < g.d - 1; ++tb) {
    int b = T[tb];
    int mine = ext_point(S, (int)q, r, grid, b, own[lane], 0);
    int sel[4], cnt = 0;
    double nodes[4];
    for (int m = 0; m < 8; ++m) {
      int jm = __shfl(mine, m, EXG);
      if (jm >= 0 && cnt < p) {
        sel[cnt] = jm;
        nodes[cnt] = (double)own[m];
        ++cnt;
      }
    }
    if (cnt < p) continue;
    double w[4];
    lagrange(0.0, nodes, p, w);
    double L = 0.0;
    for (int j = 0; j < p; ++j) L = L + fabs(w[j]);
    if (!have || L < bestL) {
      have = true;
      bestL = L;
      for (int j = 0; j < p; ++j) {
        bsel[j] = sel[j];
        bw[j] = w[j];
      }
    }
  }
  if (lane != 0) return;
  if (!have) {
    atomicOr(a.flags, FLAG_UNRESOLVED_EXT);
    for (int j = 0; j < p; ++j) {
      oi[j] = -1;
      ow[j] = 0.0;
    }
    return;
  }
  for (int j = 0; j < p; ++j) {
    oi[j] = a.s2d[bsel[j]];
    ow[j] = bw[j];
  }
}

// ---------------------------------------------------------------- irregular nodes
__device__ __forceinline__ bool in_stencil(int order, int o0, int o1, int o2) {
  if (o0 == 0 && o1 == 0 && o2 == 0) return false;
  if (order == 2) return (o0 != 0) + (o1 != 0) + (o2 != 0) == 1;
  return true;
}

struct IrrPred {
  GridDesc g;
  const int8_t* region;
  __device__ bool operator()(int64_t i) const {
    int c[3];
    unravel(g, i, c);
    for (int ax = 0; ax < g.d; ++ax)
      if (c[ax] < 1 || c[ax] > g.N - 1) return false;
    int rp = region[i];
    int zr = g.d == 3 ? 1 : 0;
    for (int o2 = -zr; o2 <= zr; ++o2)
      for (int o1 = -1; o1 <= 1; ++o1)
        for (int o0 = -1; o0 <= 1; ++o0) {
          if (!in_stencil(g.order, o0, o1, o2)) continue;
          int q[3] = {c[0] + o0, c[1] + o1, c[2] + o2};
          if (region[ravel(g, q)] != rp) return true;
        }
    return false;
  }
};

struct IdxEmit {
  int* out;
  __device__ void operator()(int64_t i, int o) const { out[o] = (int)i; }
};

__global__ void k_need_irr(GridDesc g, int64_t n_irr, const int* irr, const int8_t* region,
                           uint8_t* need) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_irr) return;
  int64_t P = irr[t];
  int c[3];
  unravel(g, P, c);
  int rp = region[P];
  int zr = g.d == 3 ? 1 : 0;
  for (int o2 = -zr; o2 <= zr; ++o2)
    for (int o1 = -1; o1 <= 1; ++o1)
      for (int o0 = -1; o0 <= 1; ++o0) {
        if (!in_stencil(g.order, o0, o1, o2)) continue;
        int q[3] = {c[0] + o0, c[1] + o1, c[2] + o2};
        int64_t Q = ravel(g, q);
        int rq = region[Q];
        if (rq == rp) continue;
        if (rp != 0) need[(int64_t)(rp - 1) * g.n_nodes + Q] = 1;
        if (rq != 0) need[(int64_t)(rq - 1) * g.n_nodes + Q] = 1;
      }
}

__device__ __forceinline__ int block_start(const GridDesc& g, double x) {
  int q = g.p;
  int st = (int)floor((x - g.lo) / g.h + 0.5) - q / 2;
  if (st < 0) st = 0;
  if (st > g.N - q) st = g.N - q;
  return st;
}

// correction entries needed by the interpolation blocks: for every centre
// (a primary candidate, before the surface table is compacted) the nodes of
// its (q+1)^d block that lie inside another interface need that
// interface's correction (the centre's own side uses its own polynomial)
__global__ void k_need_blocks_cand(GridDesc g, int64_t nc, const int* acc, const int* r, const int* ck,
                                   const double* cpos, const double* cnrm, const int8_t* region, uint8_t* need) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc || !acc[i] || !cand_primary(g.d, cnrm, r, i)) return;
  int k = ck[i];
  int st[3] = {0, 0, 0};
  for (int ax = 0; ax < g.d; ++ax) st[ax] = block_start(g, cpos[i * g.d + ax]);
  int q1 = g.p + 1;
  int nz = g.d == 3 ? q1 : 1;
  for (int b2 = 0; b2 < nz; ++b2)
    for (int b1 = 0; b1 < q1; ++b1)
      for (int b0 = 0; b0 < q1; ++b0) {
        int cc[3] = {st[0] + b0, st[1] + b1, st[2] + b2};
        int64_t Q = ravel(g, cc);
        int rq = region[Q];
        if (rq != k && rq != 0) need[(int64_t)(rq - 1) * g.n_nodes + Q] = 1;
      }
}

struct NeedPred {
  const uint8_t* need;
  __device__ bool operator()(int64_t i) const { return need[i] != 0; }
};

struct CorrEmit {
  int64_t n_nodes;
  int *k, *node;
  __device__ void operator()(int64_t i, int o) const {
    k[o] = (int)(i / n_nodes) + 1;
    node[o] = (int)(i % n_nodes);
  }
};

// ---------------------------------------------------------------- closest centres
struct BinArgs {
  GridDesc g;
  int64_t n_dof, nca, ncell;
  const int* d2s;
  const double* spos;
  const int* meta;
  int* cnt;
  int* items;
};

__device__ __forceinline__ int64_t bin_of(const GridDesc& g, int64_t nca, const double* x, int k,
                                          int64_t ncell, int cc[3]) {
  double cs = 2.0 * g.h;
  for (int ax = 0; ax < 3; ++ax) cc[ax] = 0;
  for (int ax = 0; ax < g.d; ++ax) {
    int v = (int)floor((x[ax] - g.lo) / cs);
    if (v < 0) v = 0;
    if (v > nca - 1) v = (int)nca - 1;
    cc[ax] = v;
  }
  int64_t cell = cc[0] + nca * (cc[1] + (g.d == 3 ? nca * cc[2] : 0));
  return (int64_t)(k - 1) * ncell + cell;
}

__global__ void k_bin_count(BinArgs a) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n_dof) return;
  int s = a.d2s[c];
  int cc[3];
  int64_t key = bin_of(a.g, a.nca, a.spos + (int64_t)s * a.g.d, a.meta[(int64_t)s * 5 + 3], a.ncell, cc);
  atomicAdd(a.cnt + key, 1);
}

__global__ void k_bin_fill(BinArgs a, const int* start, int* cursor) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n_dof) return;
  int s = a.d2s[c];
  int cc[3];
  int64_t key = bin_of(a.g, a.nca, a.spos + (int64_t)s * a.g.d, a.meta[(int64_t)s * 5 + 3], a.ncell, cc);
  int pos = start[key] + atomicAdd(cursor + key, 1);
  a.items[pos] = (int)c;
}

struct OwnerArgs {
  GridDesc g;
  int64_t n_corr, nca, ncell;
  const int *ck, *cnode;
  const int* d2s;
  const double* spos;
  const int *start, *cnt, *items;
  int* owner;
  int* flags;
};

constexpr int OWG = 16;   // lanes per correction entry

// cell of the (2m+1)^d box around cq with linear index idx, if it lies on
// ring m (Chebyshev distance m) and inside the grid of bins
__device__ __forceinline__ bool ring_cell(const GridDesc& g, int64_t nca, const int cq[3], int m, int idx,
                                          int64_t koff, int64_t* key) {
  const int w = 2 * m + 1;
  int o[3] = {idx % w - m, (idx / w) % w - m, g.d == 3 ? idx / (w * w) - m : 0};
  int cheb = 0;
  for (int t = 0; t < 3; ++t) {
    int v = o[t] < 0 ? -o[t] : o[t];
    cheb = v > cheb ? v : cheb;
  }
  if (cheb != m) return false;
  int cc[3] = {cq[0] + o[0], cq[1] + o[1], cq[2] + o[2]};
  for (int t = 0; t < g.d; ++t)
    if (cc[t] < 0 || cc[t] >= nca) return false;
  *key = koff + cc[0] + nca * (cc[1] + (g.d == 3 ? nca * cc[2] : 0));
  return true;
}

// Closest centre of every correction entry, one group of OWG lanes per
// entry: rings of bins are scanned in parallel (lanes over the cells of a
// ring); the same stop rule and tie rule as a sequential scan, so the owner
// is identical.
__global__ void __launch_bounds__(KFBI_BLOCK) k_owner(OwnerArgs a) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t e = t / OWG;
  int lane = (int)(t % OWG);
  if (e >= a.n_corr) return;
  const GridDesc& g = a.g;
  int k = a.ck[e];
  int c[3];
  unravel(g, a.cnode[e], c);
  double X[3] = {node_x(g, c[0]), node_x(g, c[1]), g.d == 3 ? node_x(g, c[2]) : 0.0};
  int cq[3];
  bin_of(g, a.nca, X, k, a.ncell, cq);
  int64_t koff = (int64_t)(k - 1) * a.ncell;
  double cs = 2.0 * g.h;
  double d2min = INFINITY;
  int mfinal = -1;
  for (int m = 0; m <= a.nca; ++m) {
    const int w = 2 * m + 1;
    const int ncells = g.d == 3 ? w * w * w : w * w;
    double loc = INFINITY;
    for (int idx = lane; idx < ncells; idx += OWG) {
      int64_t key;
      if (!ring_cell(g, a.nca, cq, m, idx, koff, &key)) continue;
      for (int j = a.start[key]; j < a.start[key] + a.cnt[key]; ++j) {
        const double* P = a.spos + (int64_t)a.d2s[a.items[j]] * g.d;
        double dx = X[0] - P[0], dy = X[1] - P[1];
        double d2 = dx * dx + dy * dy;
        if (g.d == 3) {
          double dz = X[2] - P[2];
          d2 = d2 + dz * dz;
        }
        loc = d2 < loc ? d2 : loc;
      }
    }
    for (int off = OWG / 2; off > 0; off >>= 1) {
      double o = __shfl_xor(loc, off, OWG);
      loc = o < loc ? o : loc;
    }
    d2min = loc < d2min ? loc : d2min;
    double lim = (double)m * cs;
    if (d2min < INFINITY && d2min * (1.0 + TIE_BAND) < lim * lim) {
      mfinal = m;
      break;
    }
  }
  if (!(d2min < INFINITY)) {
    if (lane == 0) {
      atomicOr(a.flags, FLAG_UNRESOLVED_OWNER);
      a.owner[e] = 0;
    }
    return;
  }
  if (mfinal < 0) mfinal = (int)a.nca;
  const double thr = d2min * (1.0 + TIE_BAND);
  int best = 0x7fffffff;
  for (int m = 0; m <= mfinal; ++m) {
    const int w = 2 * m + 1;
    const int ncells = g.d == 3 ? w * w * w : w * w;
    for (int idx = lane; idx < ncells; idx += OWG) {
      int64_t key;
      if (!ring_cell(g, a.nca, cq, m, idx, koff, &key)) continue;
      for (int j = a.start[key]; j < a.start[key] + a.cnt[key]; ++j) {
        const int ctr = a.items[j];
        const double* P = a.spos + (int64_t)a.d2s[ctr] * g.d;
        double dx = X[0] - P[0], dy = X[1] - P[1];
        double d2 = dx * dx + dy * dy;
        if (g.d == 3) {
          double dz = X[2] - P[2];
          d2 = d2 + dz * dz;
        }
        if (d2 <= thr && ctr < best) best = ctr;
      }
    }
  }
  for (int off = OWG / 2; off > 0; off >>= 1) {
    int o = __shfl_xor(best, off, OWG);
    best = o < best ? o : best;
  }
  if (lane == 0) a.owner[e] = best;
}

// ---------------------------------------------------------------- resets
// Up to 12 device arrays set to a value in one launch: int arrays to v, byte
// arrays (v = 0 only) to zero.  blockIdx.y selects the array.
struct FillItem {
  void* p;
  int64_t n;
  int v;
  int bytes;   // 1: uint8 elements (zeroed), 0: int elements
};
struct FillList {
  FillItem it[12];
  int n;
  void add(int* p, int64_t cnt, int v) { it[n++] = FillItem{p, cnt, v, 0}; }
  void add_bytes(uint8_t* p, int64_t cnt) { it[n++] = FillItem{p, cnt, 0, 1}; }
};

__global__ void k_fill_many(FillList L) {
  const FillItem f = L.it[blockIdx.y];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (f.bytes) {
    // whole 32-bit words, then the tail bytes (allocations are 256-byte aligned)
    uint32_t* w = (uint32_t*)f.p;
    const int64_t nw = f.n >> 2;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw; i += stride) w[i] = 0u;
    if (blockIdx.x == 0 && threadIdx.x < (f.n & 3)) ((uint8_t*)f.p)[(nw << 2) + threadIdx.x] = 0;
  } else {
    int* a = (int*)f.p;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < f.n; i += stride) a[i] = f.v;
  }
}

// ---------------------------------------------------------------- host helpers
inline unsigned nblk(int64_t n, int b = KFBI_BLOCK) { return (unsigned)((n + b - 1) / b); }

template <class T>
kfbi_status grow(T** p, int64_t* cap, int64_t n) {
  if (n <= *cap && *p) return KFBI_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  int64_t c = kfbi_headroom(n);
  if (hipMalloc((void**)p, (size_t)c * sizeof(T)) != hipSuccess) {
    *cap = 0;
    kfbi_set_error("device allocation of %lld bytes failed", (long long)(c * sizeof(T)));
    return KFBI_E_OOM;
  }
  *cap = c;
  return KFBI_OK;
}

// (re)allocate exactly n elements (contents discarded)
template <class T>
kfbi_status realloc_n(T** p, int64_t n) {
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

inline int64_t headroom(int64_t n) { return kfbi_headroom(n); }

kfbi_status ensure_blk(kfbi_plan* pl, int64_t nb) { return grow(&pl->blk, &pl->cap_blk, nb + 1); }

// the scanned total (and, if flags is given, the status flags) to the host
kfbi_status post_count(kfbi_plan* pl, int64_t* count, int* flags) {
  PostReq q{};
  q.ni = flags ? 2 : 1;
  q.isrc[0] = pl->blk_total;
  q.isrc[1] = pl->d_flags;
  int v[2] = {0, 0};
  KCHK(kfbi_post_wait(pl, q, v, nullptr));
  *count = v[0];
  if (flags) *flags = v[1];
  return KFBI_OK;
}

template <class Pred>
kfbi_status compact_count(kfbi_plan* pl, int64_t n, Pred pred, int64_t* count, int* flags = nullptr) {
  int64_t nb = (n + CMP_CH - 1) / CMP_CH;
  if (nb == 0) {
    *count = 0;
    if (flags) *flags = 0;
    return KFBI_OK;
  }
  KCHK(ensure_blk(pl, nb));
  hipLaunchKernelGGL(k_count<Pred>, dim3((unsigned)nb), dim3(KFBI_BLOCK), 0, pl->stream, n, pred, pl->blk);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, pl->stream, pl->blk, nb, pl->blk_total);
  return post_count(pl, count, flags);
}

template <class Pred>
kfbi_status compact_count_flags(kfbi_plan* pl, int64_t n, Pred pred, int64_t* count, int* flags = nullptr) {
  int64_t nb = (n + CMP_CH - 1) / CMP_CH;
  if (nb == 0) {
    *count = 0;
    if (flags) *flags = 0;
    return KFBI_OK;
  }
  KCHK(ensure_blk(pl, nb));
  hipLaunchKernelGGL(k_count_flags<Pred>, dim3((unsigned)nb), dim3(KFBI_BLOCK), 0, pl->stream, n, pred, pl->blk,
                     pl->flags8);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, pl->stream, pl->blk, nb, pl->blk_total);
  return post_count(pl, count, flags);
}

// count (storing the predicate in flags) and scan into blk, total -> *tot,
// without a host wait
template <class Pred>
void enqueue_count_flags(kfbi_plan* pl, int64_t n, Pred pred, int* blk, uint8_t* flags, int* tot) {
  const int64_t nb = (n + CMP_CH - 1) / CMP_CH;
  hipLaunchKernelGGL(k_count_flags<Pred>, dim3((unsigned)nb), dim3(KFBI_BLOCK), 0, pl->stream, n, pred, blk, flags);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, pl->stream, blk, nb, tot);
}

template <class Pred>
void enqueue_count(kfbi_plan* pl, int64_t n, Pred pred, int* blk, int* tot) {
  const int64_t nb = (n + CMP_CH - 1) / CMP_CH;
  hipLaunchKernelGGL(k_count<Pred>, dim3((unsigned)nb), dim3(KFBI_BLOCK), 0, pl->stream, n, pred, blk);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, pl->stream, blk, nb, tot);
}

template <class Pred, class Emit>
void compact_emit_with(kfbi_plan* pl, int64_t n, Pred pred, Emit emit, int* blk) {
  int64_t nb = (n + CMP_CH - 1) / CMP_CH;
  if (nb == 0) return;
  hipLaunchKernelGGL((k_emit<Pred, Emit>), dim3((unsigned)nb), dim3(KFBI_BLOCK), 0, pl->stream, n, pred, emit, blk);
}

template <class Pred, class Emit>
void compact_emit(kfbi_plan* pl, int64_t n, Pred pred, Emit emit) {
  int64_t nb = (n + CMP_CH - 1) / CMP_CH;
  if (nb == 0) return;
  hipLaunchKernelGGL((k_emit<Pred, Emit>), dim3((unsigned)nb), dim3(KFBI_BLOCK), 0, pl->stream, n, pred,
                     emit, pl->blk);
}

// lattice of degree m in D dims (D <= 2), stacking offsets 0, +1, -1, ...
void lattice(int D, int m, std::vector<std::array<int, 3>>& out) {
  out.clear();
  if (m < 0) return;
  auto window = [](int L, std::vector<int>& w) {
    w.clear();
    int a = -((L - 1) / 2);
    for (int i = 0; i < L; ++i) w.push_back(a + i);
  };
  auto stack = [](int j) { return j == 0 ? 0 : (j % 2 == 1 ? (j + 1) / 2 : -(j / 2)); };
  std::vector<int> w;
  if (D == 1) {
    window(m + 1, w);
    for (int o : w) out.push_back({o, 0, 0});
    return;
  }
  for (int j = 0; j <= m; ++j) {
    window(m - j + 1, w);
    for (int o : w) out.push_back({o, stack(j), 0});
  }
}

void shift_list(int d, const std::vector<std::array<int, 3>>& offs, int (*sh)[2], int* n) {
  std::vector<std::array<int, 2>> cand;
  if (d == 2) {
    int c[9] = {0, 1, -1, 2, -2, 3, -3, 4, -4};
    for (int v : c) cand.push_back({v, 0});
  } else {
    for (int a = -4; a <= 4; ++a)
      for (int b = -4; b <= 4; ++b) cand.push_back({a, b});
    std::stable_sort(cand.begin(), cand.end(), [](const std::array<int, 2>& s, const std::array<int, 2>& t) {
      int ks0 = std::abs(s[0]) + std::abs(s[1]), kt0 = std::abs(t[0]) + std::abs(t[1]);
      if (ks0 != kt0) return ks0 < kt0;
      if (std::abs(s[1]) != std::abs(t[1])) return std::abs(s[1]) < std::abs(t[1]);
      if (s[0] != t[0]) return s[0] > t[0];
      return s[1] > t[1];
    });
  }
  *n = 0;
  for (auto& s : cand) {
    bool member = false;
    for (auto& o : offs)
      if (o[0] == -s[0] && (d == 2 || o[1] == -s[1])) member = true;
    if (member) {
      sh[*n][0] = s[0];
      sh[*n][1] = s[1];
      ++*n;
    }
  }
}

}  // namespace

// ---------------------------------------------------------------- S0 driver
kfbi_status geo_setup(kfbi_plan* pl) {
  GridDesc g = pl->g;
  hipStream_t st = pl->stream;
  LSet L;
  bool sampled = false;
  for (int k = 0; k < g.K; ++k) sampled = sampled || pl->prob.iface[k].kind == KFBI_LS_GRID;
  if (sampled && !pl->ls_samples) {
    if (hipMalloc((void**)&pl->ls_samples, sizeof(double) * (size_t)g.K * g.n_nodes) != hipSuccess) {
      (void)hipGetLastError();
      pl->ls_samples = nullptr;
      kfbi_set_error("device allocation of the level-set samples failed");
      return KFBI_E_OOM;
    }
  }
  L.K = g.K;
  L.lo = g.lo;
  L.h = g.h;
  L.N = g.N;
  L.d = g.d;
  for (int k = 0; k < g.K; ++k) {
    L.kind[k] = pl->prob.iface[k].kind;
    for (int j = 0; j < KFBI_LS_NPARAM; ++j) L.p[k][j] = pl->prob.iface[k].p[j];
    L.S[k] = nullptr;
    if (L.kind[k] == KFBI_LS_GRID) {
      // the plan's own copy of the samples (the caller's may go away)
      double* dst = pl->ls_samples + (int64_t)k * g.n_nodes;
      HIPCHK(hipMemcpyAsync(dst, pl->prob.samples[k], sizeof(double) * g.n_nodes, hipMemcpyDeviceToDevice, st));
      L.S[k] = dst;
    }
  }
  // every grid-sized table that the set-up fills sparsely starts from its
  // reset value: one launch instead of a memset each
  {
    const int64_t nkeys = (int64_t)g.K * pl->ncell;
    const int64_t nrows = g.d == 3 ? (int64_t)g.n1 * g.n1 : g.n1;
    FillList F;
    F.n = 0;
    F.add(pl->d_flags, 1, 0);
    F.add(pl->line_start, pl->n_lines, 0);
    F.add(pl->line_end, pl->n_lines, 0);
    F.add(pl->cell_count, nkeys + 1, 0);
    F.add(pl->cell_cursor, nkeys + 1, 0);
    F.add(pl->EI, (int64_t)g.K * g.n_nodes, -1);
    F.add(pl->row_start, nrows, 0);
    F.add(pl->row_end, nrows, 0);
    F.add_bytes(pl->need, (int64_t)g.K * g.n_nodes);
    int64_t most = 0;
    for (int i = 0; i < F.n; ++i) most = F.it[i].n > most ? F.it[i].n : most;
    const int64_t gx = (most + 4 * KFBI_BLOCK - 1) / (4 * KFBI_BLOCK);
    hipLaunchKernelGGL(k_fill_many, dim3((unsigned)(gx < 2048 ? gx : 2048), (unsigned)F.n), dim3(KFBI_BLOCK), 0, st, F);
  }
  // regions
  hipLaunchKernelGGL(k_regions, dim3(nblk(g.n_nodes)), dim3(KFBI_BLOCK), 0, st,
                     RegionArgs{g, L, pl->region, pl->d_flags});
  // the region flags travel with the first compaction count (one host
  // wait); the candidate count reads the regions only
  // candidates: (segment, interface) items with a sign change
  // the irregular nodes depend on the regions only: they are counted in the
  // same host wait
  int64_t n_items = pl->n_seg * g.K;
  CandPred cp{g, pl->region};
  IrrPred ip{g, pl->region};
  int64_t nc, ni;
  {
    const int64_t nbc = (n_items + CMP_CH - 1) / CMP_CH, nbi = (g.n_nodes + CMP_CH - 1) / CMP_CH;
    KCHK(ensure_blk(pl, nbc));
    KCHK(grow(&pl->blk2, &pl->cap_blk2, nbi + 1));
    enqueue_count_flags(pl, n_items, cp, pl->blk, pl->flags8, pl->blk_total);
    enqueue_count_flags(pl, g.n_nodes, ip, pl->blk2, pl->flags8b, pl->blk_total + 1);
    PostReq q{};
    q.ni = 3;
    q.isrc[0] = pl->blk_total;
    q.isrc[1] = pl->blk_total + 1;
    q.isrc[2] = pl->d_flags;
    int v[3] = {0, 0, 0};
    KCHK(kfbi_post_wait(pl, q, v, nullptr));
    nc = v[0];
    ni = v[1];
    if (v[2]) return kfbi_flags_status(v[2]);
  }
  if (ni > pl->cap_irr) {
    int64_t cap = headroom(ni);
    pl->cap_irr = 0;
    KCHK(realloc_n(&pl->irr, cap));
    pl->cap_irr = cap;
  }
  pl->n_irr = ni;
  compact_emit_with(pl, g.n_nodes, NeedPred{pl->flags8b}, IdxEmit{pl->irr}, pl->blk2);
  if (nc == 0) {
    kfbi_set_error("no grid segment crosses an interface");
    return KFBI_E_INVALID;
  }
  if (nc > pl->cap_cand) {
    int64_t cap = headroom(nc);
    pl->cap_cand = 0;
    KCHK(realloc_n(&pl->c_r, cap));
    KCHK(realloc_n(&pl->c_lid, cap));
    KCHK(realloc_n(&pl->c_seg, cap));
    KCHK(realloc_n(&pl->c_k, cap));
    KCHK(realloc_n(&pl->c_ina, cap));
    KCHK(realloc_n(&pl->c_acc, cap));
    KCHK(realloc_n(&pl->c_pos, cap * g.d));
    KCHK(realloc_n(&pl->c_nrm, cap * g.d));
    pl->cap_cand = cap;
  }
  pl->n_cand = nc;
  compact_emit(pl, n_items, NeedPred{pl->flags8},
               CandEmit{g, pl->region, pl->c_r, pl->c_lid, pl->c_seg, pl->c_k, pl->c_ina});
  hipLaunchKernelGGL(k_bisect, dim3(nblk(nc * BIS_G)), dim3(KFBI_BLOCK), 0, st,
                     BisectArgs{g, L, nc, pl->c_r, pl->c_lid, pl->c_seg, pl->c_k, pl->c_ina, pl->c_pos,
                                pl->c_nrm, pl->c_acc});

  // surface points, centres and correction entries are counted in one host
  // wait, all from the candidates: accepted ones (surface table), accepted
  // primary ones (centres), and the (interface, node) entries that the
  // irregular nodes and the centres' interpolation blocks need
  AccPred ap{pl->c_acc};
  PrimCandPred pcp{g.d, pl->c_acc, pl->c_r, pl->c_nrm};
  NeedPred np{pl->need};
  const int64_t n_need = (int64_t)g.K * g.n_nodes;
  int64_t ns, nd, ne;
  {
    const int64_t nbc = (nc + CMP_CH - 1) / CMP_CH, nbn = (n_need + CMP_CH - 1) / CMP_CH;
    KCHK(ensure_blk(pl, nbc));
    KCHK(grow(&pl->blk2, &pl->cap_blk2, nbn + 1));
    KCHK(grow(&pl->blk3, &pl->cap_blk3, nbc + 1));
    enqueue_count(pl, nc, ap, pl->blk, pl->blk_total);
    enqueue_count(pl, nc, pcp, pl->blk3, pl->blk_total + 1);
    if (ni > 0)
      hipLaunchKernelGGL(k_need_irr, dim3(nblk(ni)), dim3(KFBI_BLOCK), 0, st, g, ni, pl->irr, pl->region,
                         pl->need);
    hipLaunchKernelGGL(k_need_blocks_cand, dim3(nblk(nc)), dim3(KFBI_BLOCK), 0, st, g, nc, pl->c_acc, pl->c_r,
                       pl->c_k, pl->c_pos, pl->c_nrm, pl->region, pl->need);
    enqueue_count(pl, n_need, np, pl->blk2, pl->blk_total + 2);
    PostReq q{};
    q.ni = 3;
    for (int i = 0; i < 3; ++i) q.isrc[i] = pl->blk_total + i;
    int v[3] = {0, 0, 0};
    KCHK(kfbi_post_wait(pl, q, v, nullptr));
    ns = v[0];
    nd = v[1];
    ne = v[2];
  }
  if (ns > pl->cap_surf) {
    int64_t cap = headroom(ns);
    pl->cap_surf = 0;
    KCHK(realloc_n(&pl->s_pos, cap * g.d));
    KCHK(realloc_n(&pl->s_nrm, cap * g.d));
    KCHK(realloc_n(&pl->s_meta, cap * 5));
    KCHK(realloc_n(&pl->s2d, cap));
    KCHK(realloc_n(&pl->s_need, cap));
    KCHK(realloc_n(&pl->ext_idx, cap * g.p));
    KCHK(realloc_n(&pl->ext_w, cap * g.p));
    KCHK(realloc_n(&pl->psiS, cap));
    KCHK(realloc_n(&pl->aS, cap));
    pl->cap_surf = cap;
  }
  pl->n_surf = ns;
  compact_emit(pl, nc, ap, SurfEmit{g.d, pl->c_pos, pl->c_nrm, pl->c_r, pl->c_lid, pl->c_seg, pl->c_k,
                                    pl->s_pos, pl->s_nrm, pl->s_meta});
  int64_t L1 = g.d == 2 ? g.n1 : (int64_t)g.n1 * g.n1;
  hipLaunchKernelGGL(k_lines, dim3(nblk(ns)), dim3(KFBI_BLOCK), 0, st, ns, L1, pl->s_meta, pl->line_start,
                     pl->line_end, pl->s2d, pl->s_need);

  // primary points (their count is known: the scan over the surface table
  // only places them)
  PrimPred pp{pl->s_meta};
  if (nd == 0) {
    kfbi_set_error("no primary surface points");
    return KFBI_E_INVALID;
  }
  if (nd > pl->cap_dof) {
    int64_t cap = headroom(nd);
    pl->cap_dof = 0;
    KCHK(realloc_n(&pl->d2s, cap));
    KCHK(realloc_n(&pl->stD, cap * pl->nD));
    KCHK(realloc_n(&pl->stN, cap * pl->nN));
    KCHK(realloc_n(&pl->MinvT, cap * pl->nC * pl->nC));
    KCHK(realloc_n(&pl->MT, cap * pl->nC * pl->nC));
    KCHK(realloc_n(&pl->cond, cap));
    KCHK(realloc_n(&pl->U, cap * pl->nC));
    KCHK(realloc_n(&pl->dn_in, cap));
    KCHK(realloc_n(&pl->dn_out, cap));
    KCHK(realloc_n(&pl->bvec, cap));
    KCHK(realloc_n(&pl->work, cap));
    KCHK(realloc_n(&pl->work2, cap));
    KCHK(realloc_n(&pl->cell_items, cap));
    pl->cap_dof = cap;
  }
  pl->n_dof = nd;
  if (ns > 0) enqueue_count(pl, ns, pp, pl->blk, pl->blk_total + 3);
  compact_emit(pl, ns, pp, PrimEmit{pl->d2s, pl->s2d});

  // collocation stencils
  Lattices lat;
  std::vector<std::array<int, 3>> offs;
  lattice(g.d - 1, g.p, offs);
  lat.nD = (int)offs.size();
  for (int m = 0; m < lat.nD; ++m) {
    lat.offD[m][0] = offs[m][0];
    lat.offD[m][1] = offs[m][1];
  }
  shift_list(g.d, offs, lat.shD, &lat.nSD);
  lattice(g.d - 1, g.p - 1, offs);
  lat.nN = (int)offs.size();
  for (int m = 0; m < lat.nN; ++m) {
    lat.offN[m][0] = offs[m][0];
    lat.offN[m][1] = offs[m][1];
  }
  shift_list(g.d, offs, lat.shN, &lat.nSN);
  SurfView S{g, pl->s_pos, pl->s_nrm, pl->s_meta, pl->line_start, pl->line_end, L1};
  hipLaunchKernelGGL(k_stencils, dim3(nblk(nd * STG)), dim3(KFBI_BLOCK), 0, st,
                     StencilArgs{S, lat, nd, pl->d2s, pl->stD, pl->stN, pl->s_need, pl->d_flags});
  hipLaunchKernelGGL(k_extension, dim3(nblk(ns * EXG)), dim3(KFBI_BLOCK), 0, st,
                     ExtArgs{S, ns, pl->s2d, pl->s_need, pl->ext_idx, pl->ext_w, pl->d_flags});

  // correction entries (counted above; the scan is in blk2)
  if (ne > pl->cap_corr) {
    int64_t cap = headroom(ne);
    pl->cap_corr = 0;
    KCHK(realloc_n(&pl->ce_k, cap));
    KCHK(realloc_n(&pl->ce_node, cap));
    KCHK(realloc_n(&pl->ce_owner, cap));
    pl->cap_corr = cap;
  }
  pl->n_corr = ne;
  compact_emit_with(pl, n_need, np, CorrEmit{g.n_nodes, pl->ce_k, pl->ce_node}, pl->blk2);

  // closest centres: bin the centres of every interface on a 2h lattice
  int64_t nkeys = (int64_t)g.K * pl->ncell;
  BinArgs ba{g, nd, pl->ncell_axis, pl->ncell, pl->d2s, pl->s_pos, pl->s_meta, pl->cell_count, nullptr};
  hipLaunchKernelGGL(k_bin_count, dim3(nblk(nd)), dim3(KFBI_BLOCK), 0, st, ba);
  {
    int64_t nbs = (nkeys + CMP_CH - 1) / CMP_CH;
    KCHK(ensure_blk(pl, nbs));
    hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nbs), dim3(KFBI_BLOCK), 0, st, nkeys, pl->cell_count, pl->blk);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, pl->blk, nbs, pl->blk_total);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nbs), dim3(KFBI_BLOCK), 0, st, nkeys, pl->cell_count,
                       pl->cell_start, pl->blk);
  }
  ba.items = pl->cell_items;
  hipLaunchKernelGGL(k_bin_fill, dim3(nblk(nd)), dim3(KFBI_BLOCK), 0, st, ba, pl->cell_start, pl->cell_cursor);
  if (ne > 0)
    hipLaunchKernelGGL(k_owner, dim3(nblk(ne * OWG)), dim3(KFBI_BLOCK), 0, st,
                       OwnerArgs{g, ne, pl->ncell_axis, pl->ncell, pl->ce_k, pl->ce_node, pl->d2s, pl->s_pos,
                                 pl->cell_start, pl->cell_count, pl->cell_items, pl->ce_owner, pl->d_flags});
  // the flags of the stencil, extension and owner searches are read back with
  // the collocation's (one host wait); the factorisation skips its work when
  // one is set
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

// PDE collocation lattice (degree p-2 in d dims) for other translation units
void kfbi_pde_lattice(int d, int p, int (*off)[3], int* n) {
  std::vector<std::array<int, 3>> pts;
  int m = p - 2;
  *n = 0;
  if (m < 0) return;
  if (d == 2) {
    lattice(2, m, pts);
    for (auto& o : pts) {
      off[*n][0] = o[0];
      off[*n][1] = o[1];
      off[*n][2] = 0;
      ++*n;
    }
    return;
  }
  auto stack = [](int j) { return j == 0 ? 0 : (j % 2 == 1 ? (j + 1) / 2 : -(j / 2)); };
  for (int j = 0; j <= m; ++j) {
    lattice(2, m - j, pts);
    for (auto& o : pts) {
      off[*n][0] = o[0];
      off[*n][1] = o[1];
      off[*n][2] = stack(j);
      ++*n;
    }
  }
}

void kfbi_dn_lattice(int D, int m, int (*off)[2], int* n) {
  std::vector<std::array<int, 3>> pts;
  lattice(D, m, pts);
  *n = (int)pts.size();
  for (int i = 0; i < *n; ++i) {
    off[i][0] = pts[i][0];
    off[i][1] = pts[i][1];
  }
}
