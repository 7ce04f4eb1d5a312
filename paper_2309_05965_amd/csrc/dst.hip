// Step S3 -- box solve A_h v = F with homogeneous Dirichlet data.
//
// Paper: Alg. 1 Step 3.3 solves the corrected finite-difference system by a
// fast Fourier method; Sec. 5.2 gives the operators (eqs. 9p-cds, 27p-cds).  With
// homogeneous box data every operator of the library is diagonal in the
// type-I sine basis: per axis the 3-point second difference has eigenvalue
// s_k = -4/h^2 sin^2(k pi / 2N), k = 1..N-1, and
//   order 4: lambda = sum s + h^2/6 sum_{a<b} s_a s_b (+ h^4/48 s_x s_y s_z)
//                     - kappa (1 + h^2/12 sum s)
//   order 2: lambda = sum s - kappa.
// The unnormalised DST-I S (S_kj = sin(pi j k / N)) satisfies S^2 = N/2 I,
// so v = (2/N)^d S_d (S_d F / lambda).
//
// Design for gfx950: one HBM read and one HBM write per axis pass.  A work
// group loads a tile of TL lines (coalesced along x), forms the odd
// extension of two real lines as the real and imaginary parts of one complex
// sequence of length M = 2N, runs self-sorting Stockham FFTs (radix 4) in
// LDS ping-pong buffers, and unpacks both
// sine transforms from the result (Re Z_k = 2 S_B(k), Im Z_k = -2 S_A(k)).
// The last axis is fused: forward DST, spectral divide and inverse DST in
// LDS, so 2D takes 3 passes and 3D 5 passes of 16 B per node.  Tiles are
// dealt in XCD-contiguous order, and the tile size trades a work group's
// fixed latency against LDS residency (tile_lines).  Twiddles are read
// from a global table (L2-resident).
#include <math.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <mutex>
#include <new>
#include <vector>

#include "kfbi_internal.h"

namespace {

constexpr size_t DST_LDS_CU = 163840;  // LDS of one compute unit
constexpr int DST_CH = 8;               // loads in flight per thread while a tile is read
constexpr int PS = 3;                   // LDS pad shift (see padi)

struct DstArgs {
  const int* ctl;      // nothing to do once ctl[1] is set (device GMRES loop)
  const int* mctl;     // nor once mctl[0] is set (converged multigrid loop, coarse solves)
  // source of the first pass of the matvec: the corrected right-hand side,
  // zero except at the irregular nodes, built here from the correction
  // values of the density
  int src_corr;
  const int *row_start, *row_end, *irr, *PE1, *PE2;
  const double *PA, *Cv;
  const double* Firr;  // F at the irregular nodes, precomputed (long pair tables), or null
  int maxpairs;
  GridDesc g;
  int ax;          // transform axis
  int mode;        // 0: DST; 1: DST, divide by lambda and scale, DST
  int TL;          // lines per tile (even)
  int tiles_u;     // tiles along the tile axis
  const double* in;
  double* out;
  const double2* tw;   // exp(-2 pi i m / M), m < M
  const double* eig1;  // s_k, k = 0..N
  double scale;        // (2/N)^d
  // first pass of a multigrid coarse solve (3D, x axis): instead of reading
  // `in`, the coarse right-hand side is the full weighting of this fine
  // residual (FP32 if rsrc_f32, else FP64; n1f nodes per axis), formed on load
  const void* rsrc;
  int rsrc_f32, n1f;
};

// LDS layout of a sequence: element i at i + (i >> PS), one pad slot per 8
// 16-byte elements, so the strided writes of the early Stockham stages
// spread over the banks
__device__ __forceinline__ int padi(int i) { return i + (i >> PS); }

constexpr int padded_len(int M) { return M + (M >> PS); }

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Stockham FFT of length M = 2^LOGM: radix-4 stages s = 0..LOGM/2-1 (span
// Ns = 4^s), then one radix-2 stage if LOGM is odd.  A stage with span Ns
// reads x[j + r M/R], twiddles by exp(-2 pi i r k/(R Ns)), k = j mod Ns,
// and writes y[(j - k) R + k + r Ns].  With 256 threads, t = threadIdx.x +
// 256 i, the k of a radix-4 stage is threadIdx.x mod Ns for every i (Ns <=
// 256 for M <= 2048), so a thread's twiddles are fixed per stage and are
// read once, into registers, before the tile arrives.  Only the closing
// radix-2 stage of M = 2048 (Ns = 1024) cycles through four.
template <int LOGM>
struct Twiddles {
  static constexpr int M = 1 << LOGM, NS4 = LOGM / 2;
  static constexpr int N2 = (LOGM & 1) ? (M / 2 > KFBI_BLOCK ? M / 2 / KFBI_BLOCK : 1) : 1;
  double2 w4[NS4 > 1 ? NS4 - 1 : 1][3];   // stages 1..NS4-1 (stage 0: k = 0, unit twiddles)
  double2 w2[N2];

  __device__ __forceinline__ void load(const double2* __restrict__ tw) {
#pragma unroll
    for (int s = 1; s < NS4; ++s) {
      const int st = ((int)threadIdx.x & ((1 << (2 * s)) - 1)) << (LOGM - 2 - 2 * s);
      w4[s - 1][0] = tw[st];
      w4[s - 1][1] = tw[2 * st];
      w4[s - 1][2] = tw[3 * st];
    }
    if (LOGM & 1) {
#pragma unroll
      for (int r = 0; r < N2; ++r) w2[r] = tw[((int)threadIdx.x + KFBI_BLOCK * r) & (M / 2 - 1)];
    }
  }
};

// nf forward DFTs of length M (natural order in and out) in the LDS
// buffers a and b; returns the one that holds the result
template <int LOGM>
__device__ double2* fft_stockham(double2* a, double2* b, const Twiddles<LOGM>& T, int nf) {
  constexpr int M = 1 << LOGM, Mp = padded_len(M), NS4 = LOGM / 2;
#pragma unroll
  for (int s = 0; s < NS4; ++s) {
    const int Ns = 1 << (2 * s);
    constexpr int lQ = LOGM - 2, Q = 1 << lQ;
    for (int t = threadIdx.x; t < (nf << lQ); t += KFBI_BLOCK) {
      const int f = t >> lQ, j = t & (Q - 1), k = j & (Ns - 1);
      const double2* x = a + f * Mp;
      double2* y = b + f * Mp;
      double2 v0 = x[padi(j)], v1 = x[padi(j + Q)], v2 = x[padi(j + 2 * Q)], v3 = x[padi(j + 3 * Q)];
      if (s > 0) {
        v1 = cmul(v1, T.w4[s - 1][0]);
        v2 = cmul(v2, T.w4[s - 1][1]);
        v3 = cmul(v3, T.w4[s - 1][2]);
      }
      double2 t0 = make_double2(v0.x + v2.x, v0.y + v2.y), t1 = make_double2(v0.x - v2.x, v0.y - v2.y);
      double2 t2 = make_double2(v1.x + v3.x, v1.y + v3.y), t3 = make_double2(v1.x - v3.x, v1.y - v3.y);
      const int d = ((j - k) << 2) + k;
      y[padi(d)] = make_double2(t0.x + t2.x, t0.y + t2.y);
      y[padi(d + Ns)] = make_double2(t1.x + t3.y, t1.y - t3.x);
      y[padi(d + 2 * Ns)] = make_double2(t0.x - t2.x, t0.y - t2.y);
      y[padi(d + 3 * Ns)] = make_double2(t1.x - t3.y, t1.y + t3.x);
    }
    __syncthreads();
    double2* tmp = a;
    a = b;
    b = tmp;
  }
  if (LOGM & 1) {
    // span Ns = M/2: k = j, output positions j and j + M/2
    constexpr int lQ = LOGM - 1, Q = 1 << lQ, N2 = Twiddles<LOGM>::N2;
    for (int t0 = threadIdx.x; t0 < (nf << lQ); t0 += KFBI_BLOCK * N2) {
#pragma unroll
      for (int r = 0; r < N2; ++r) {
        const int t = t0 + KFBI_BLOCK * r;
        if (t >= (nf << lQ)) break;
        const int f = t >> lQ, j = t & (Q - 1);
        const double2* x = a + f * Mp;
        double2* y = b + f * Mp;
        const double2 v0 = x[padi(j)], v1 = cmul(x[padi(j + Q)], T.w2[r]);
        y[padi(j)] = make_double2(v0.x + v1.x, v0.y + v1.y);
        y[padi(j + Q)] = make_double2(v0.x - v1.x, v0.y - v1.y);
      }
    }
    __syncthreads();
    double2* tmp = a;
    a = b;
    b = tmp;
  }
  return a;
}

// ---------------------------------------------------------------- four-step FFT, M = 1024
// One sequence per work group (TL = 2) of length 1024 = 16 x 64, x[64 n1 +
// n2] -> X[k1 + 16 k2]: 64 DFTs of length 16 over n1, a quad of lanes per
// n2 (each lane a radix-4 over n1 = c + 4m, then a radix-4 across the quad
// exchanged by DPP), the twiddle w^(n2 k1), one transpose through LDS, then
// 16 DFTs of length 64 over n2, a 16-lane row per k1 (each lane a radix-4
// over n2 = d + 16m, then a 16-point DFT across the row as two radix-4
// steps exchanged by DPP).  Each cross-lane radix-4 is two radix-2 steps
// with one exchange each, its outputs in bit-reversed lane order.  Two LDS round trips and two barriers instead of
// the five of the radix-4 Stockham stages; w = exp(-2 pi i / 1024).
constexpr int DPP_QX1 = 0xB1, DPP_QX2 = 0x4E, DPP_QX3 = 0x1B;   // quad_perm: lane i ^ 1, i ^ 2, i ^ 3
constexpr int DPP_ROR8 = 0x128;                                 // row_ror:8: lane i ^ 8 of the row
constexpr int DPP_HMIRROR = 0x141;                              // row_half_mirror: lane i ^ 7 of the row

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)u, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int CTRL>
__device__ __forceinline__ double2 dpp2(double2 v) {
  return make_double2(dpp_d<CTRL>(v.x), dpp_d<CTRL>(v.y));
}

// radix-4 DFT of four values held by one lane, natural order
__device__ __forceinline__ void dft4(double2 (&v)[4]) {
  const double2 s0 = make_double2(v[0].x + v[2].x, v[0].y + v[2].y), d0 = make_double2(v[0].x - v[2].x, v[0].y - v[2].y);
  const double2 s1 = make_double2(v[1].x + v[3].x, v[1].y + v[3].y), d1 = make_double2(v[1].x - v[3].x, v[1].y - v[3].y);
  v[0] = make_double2(s0.x + s1.x, s0.y + s1.y);
  v[1] = make_double2(d0.x + d1.y, d0.y - d1.x);
  v[2] = make_double2(s0.x - s1.x, s0.y - s1.y);
  v[3] = make_double2(d0.x - d1.y, d0.y + d1.x);
}

// radix-2 step between a lane and its partner u (the DPP-exchanged value):
// the lower lane of the pair keeps v + u, the upper one u - v (a multiply
// by -1 is exact, so both are the correctly rounded sum / difference)
__device__ __forceinline__ double2 bfly(double2 v, double2 u, bool upper) {
  const double sg = upper ? -1.0 : 1.0;
  return make_double2(fma(v.x, sg, u.x), fma(v.y, sg, u.y));
}

// v (-i) where m
__device__ __forceinline__ double2 mi_if(double2 v, bool m) { return m ? make_double2(v.y, -v.x) : v; }

// a 4-point DFT across the lanes g = 0..3 of a group as two radix-2 steps
// (partners g ^ 2, then g ^ 1); lane g ends with output bit-reversed g
__device__ __forceinline__ int brev2(int g) { return ((g & 1) << 1) | (g >> 1); }

// the thread's fixed twiddles
struct Tw4 {
  double2 q[3];   // w^(64 c k), k = 1..3
  double2 t[4];   // w^(n2 (k + 4 brev2(c))), k = 0..3
  double2 r[3];   // w^(16 d k), k = 1..3
  double2 s;      // w^(64 d0 brev2(d1))
  __device__ __forceinline__ void load(const double2* __restrict__ tw) {
    const int th = threadIdx.x, n2 = th >> 2, c = th & 3, d = th & 15;
#pragma unroll
    for (int k = 1; k < 4; ++k) {
      q[k - 1] = tw[64 * c * k];
      r[k - 1] = tw[16 * d * k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) t[k] = tw[n2 * (k + 4 * brev2(c))];
    s = tw[64 * (d & 3) * brev2(d >> 2)];
  }
};

// the output index of value q (0..3) of this thread after step 2
__device__ __forceinline__ int fs_out_index(int q) {
  const int th = threadIdx.x, k1 = th >> 4, d = th & 15;
  return k1 + 16 * (q + 4 * (brev2(d >> 2) + 4 * brev2(d & 3)));
}

// forward DFT of the 1024-point sequence whose elements 64 (c + 4m) + n2,
// m = 0..3, this thread holds in v (n2 = thread / 4, c = thread mod 4); x
// is the LDS transpose buffer; y[q] = X[fs_out_index(q)].  Ends with no
// barrier after the reads of x.
__device__ __forceinline__ void fft1024_regs(double2 (&v)[4], double2* x, const Tw4& T, double2 (&y)[4]) {
  const int th = threadIdx.x;
  {
    const int n2 = th >> 2, c = th & 3;
    dft4(v);
#pragma unroll
    for (int k = 1; k < 4; ++k) v[k] = cmul(v[k], T.q[k - 1]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double2 z = mi_if(bfly(v[k], dpp2<DPP_QX2>(v[k]), c & 2), c == 3);
      z = bfly(z, dpp2<DPP_QX1>(z), c & 1);
      x[padi(64 * (k + 4 * brev2(c)) + n2)] = cmul(z, T.t[k]);
    }
  }
  __syncthreads();
  {
    const int k1 = th >> 4, d = th & 15, d0 = d & 3, d1 = d >> 2;
#pragma unroll
    for (int m = 0; m < 4; ++m) v[m] = x[padi(64 * k1 + d + 16 * m)];
    dft4(v);
#pragma unroll
    for (int k = 1; k < 4; ++k) v[k] = cmul(v[k], T.r[k - 1]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      // across d1 (row lanes d ^ 8, then d ^ 4 = half mirror, quad ^ 3), then
      // across d0 (the quad: ^ 2, then ^ 1)
      double2 z = mi_if(bfly(v[k], dpp2<DPP_ROR8>(v[k]), d1 & 2), d1 == 3);
      z = bfly(z, dpp2<DPP_QX3>(dpp2<DPP_HMIRROR>(z)), d1 & 1);
      z = cmul(z, T.s);
      z = mi_if(bfly(z, dpp2<DPP_QX2>(z), d0 & 2), d0 == 3);
      y[k] = bfly(z, dpp2<DPP_QX1>(z), d0 & 1);
    }
  }
}

// address of element j (0..N along the axis) of the line at tile
// coordinate u and remaining coordinate w
__device__ __forceinline__ int64_t elem_addr(const DstArgs& a, int u, int w, int j) {
  const GridDesc& g = a.g;
  int c[3] = {0, 0, 0};
  c[a.ax] = j;
  int ua = a.ax == 0 ? 1 : 0;                      // tile axis
  c[ua] = u;
  if (g.d == 3) {
    int wa = 3 - a.ax - ua;                        // remaining axis
    c[wa] = w;
  }
  return (int64_t)c[0] + (int64_t)g.n1 * ((int64_t)c[1] + (int64_t)g.n1 * c[2]);
}

// full weighting at coarse node (I0, I1, I2) of the fine residual r (3D):
// the tensor product of (1/4, 1/2, 1/4) about fine node 2I, summed in T with
// o0 fastest
template <typename T>
__device__ __forceinline__ T restrict_fine(const T* __restrict__ r, int n1f, int I0, int I1, int I2) {
  const T w1[3] = {(T)0.25, (T)0.5, (T)0.25};
  T s = 0;
#pragma unroll
  for (int o2 = -1; o2 <= 1; ++o2)
#pragma unroll
    for (int o1 = -1; o1 <= 1; ++o1)
#pragma unroll
      for (int o0 = -1; o0 <= 1; ++o0) {
        T w = w1[o0 + 1] * w1[o1 + 1];
        w *= w1[o2 + 1];
        const int64_t fi = (2 * I0 + o0) + (int64_t)n1f * ((2 * I1 + o1) + (int64_t)n1f * (2 * I2 + o2));
        s += w * r[fi];
      }
  return s;
}

// lambda from the 1D eigenvalues s_k (k along the transform axis), s_u and,
// in 3D, s_w
__device__ __forceinline__ double eigenvalue(const GridDesc& g, double sk, double su, double sw) {
  const double h2 = g.h * g.h;
  double lap, pr, tri = 0.0;
  if (g.d == 2) {
    lap = sk + su;
    pr = sk * su;
  } else {
    lap = sk + su + sw;
    pr = sk * su + sk * sw + su * sw;
    tri = sk * su * sw;
  }
  if (g.order == 2) return lap - g.kappa;
  double lam = lap + h2 / 6.0 * pr;
  if (g.d == 3) lam += h2 * h2 / 48.0 * tri;
  return lam - g.kappa * (1.0 + h2 / 12.0 * lap);
}

// tile element idx -> line l (0..TL-1) and position j (1..N-1) along the
// transform axis, ordered so that consecutive threads touch consecutive
// addresses (along the line for the x axis, across the tile's lines else)
__device__ __forceinline__ void tile_pos(const DstArgs& a, int idx, int nl, int& l, int& j) {
  if (a.ax == 0) {
    j = idx % nl + 1;
    l = idx / nl;
  } else {
    l = idx % a.TL;
    j = idx / a.TL + 1;
  }
}

// F at the irregular nodes of the tile's rows: minus the sum over cut
// neighbours Q of A_PQ (C^(reg P) - C^(reg Q))(x_Q), from the correction
// values of the current density; zero elsewhere.  The pair table of a node
// is read four pairs at a time so that the gathers of a group are in flight
// together; the sum runs over the pairs in table order.
template <int M>
__device__ void corrected_rhs(const DstArgs& a, double2* A, int u0, int w) {
  const GridDesc& g = a.g;
  constexpr int Mp = padded_len(M);
  const int nl = g.N - 1, nf = a.TL / 2;
  for (int i = threadIdx.x; i < nf * Mp; i += blockDim.x) A[i] = make_double2(0.0, 0.0);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int l = wave; l < a.TL; l += nw) {
    const int u = u0 + l;
    if (u > nl) continue;
    const int64_t row = (int64_t)u + (int64_t)g.n1 * (g.d == 3 ? w : 0);
    const int r0 = a.row_start[row], r1 = a.row_end[row];
    for (int t = r0 + lane; t < r1; t += 64) {
      double F = 0.0;
      const int64_t base = (int64_t)t * a.maxpairs;
      if (a.Firr) F = a.Firr[t];
      for (int m0 = 0; !a.Firr && m0 < a.maxpairs; m0 += 4) {
        double cf[4], c1[4], c2[4];
        int e1[4], e2[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const bool in = m0 + q < a.maxpairs;
          cf[q] = in ? a.PA[base + m0 + q] : 0.0;
          e1[q] = in ? a.PE1[base + m0 + q] : -1;
          e2[q] = in ? a.PE2[base + m0 + q] : -1;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          c1[q] = e1[q] >= 0 ? a.Cv[e1[q]] : 0.0;
          c2[q] = e2[q] >= 0 ? a.Cv[e2[q]] : 0.0;
        }
        bool done = false;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          done = done || cf[q] == 0.0;      // the table is zero-padded after the last pair
          if (!done) F -= cf[q] * (c1[q] - c2[q]);
        }
        if (done) break;
      }
      const int j = a.irr[t] % g.n1;
      double2* z = A + (l >> 1) * Mp;
      if (l & 1) {
        z[padi(j)].y = F;
        z[padi(M - j)].y = -F;
      } else {
        z[padi(j)].x = F;
        z[padi(M - j)].x = -F;
      }
    }
  }
}

// LDS of a work group: the two ping-pong buffers
size_t tile_lds(int TL, int N) { return sizeof(double2) * 2 * (size_t)(TL / 2) * padded_len(2 * N); }

// One axis pass (MODE 0: DST; MODE 1: DST, divide by lambda and scale, DST):
// a work group transforms one tile of TL lines, FFT length M = 2N =
// 2^LOGM.  Every global load the tile needs -- the input, the thread's
// twiddles and (MODE 1) the 1D eigenvalues -- is issued up front, so the
// work group waits on HBM once before its FFT stages.
template <int LOGM, int MODE, bool FS>
__device__ __forceinline__ void dst_pass(const DstArgs& a, const int tile) {
  static_assert(!FS || (LOGM == 10 && MODE == 0), "the four-step FFT is written for M = 1024, one transform");
  // a converged multigrid loop skips most of its coarse solves: tested
  // before any load
  if (a.mctl && a.mctl[0]) return;
  // the GMRES converged flag is read first but tested only once the tile's
  // loads are in flight, so its latency overlaps theirs (a skipped pass has
  // only read and staged in LDS)
  const int stop = a.ctl ? a.ctl[1] : 0;
  constexpr int M = 1 << LOGM, N = M / 2, Mp = padded_len(M);
  extern __shared__ double2 lds[];
  const GridDesc& g = a.g;
  const int TL = a.TL, nf = TL / 2;
  double2* A = lds;                                 // [nf][Mp]
  double2* B = lds + nf * Mp;                       // [nf][Mp]
  const int w = tile / a.tiles_u + 1;               // remaining interior coordinate (3D)
  const int u0 = 1 + (tile % a.tiles_u) * TL;       // first tile coordinate
  constexpr int nl = N - 1;
  const int total = TL * nl;
  Twiddles<LOGM> T;
  Tw4 T4;
  if constexpr (FS)
    T4.load(a.tw);
  else
    T.load(a.tw);
  // MODE 1: s_k for this thread's k = threadIdx.x + 256 q, s_u of the
  // tile's lines and s_w
  constexpr int NE = MODE == 1 ? (N + KFBI_BLOCK - 1) / KFBI_BLOCK : 1;
  double sk[NE], su[8], sw = 0.0;
  if (MODE == 1) {
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int k = threadIdx.x + q * KFBI_BLOCK;
      sk[q] = k <= nl ? a.eig1[k] : 0.0;
    }
#pragma unroll
    for (int l = 0; l < 8; ++l) su[l] = a.eig1[(l < TL && u0 + l <= nl) ? u0 + l : 1];
    if (g.d == 3) sw = a.eig1[w];
  }
  if (a.src_corr) {
    corrected_rhs<M>(a, A, u0, w);
  } else {
    for (int f = threadIdx.x; f < nf; f += blockDim.x) {
      A[f * Mp] = make_double2(0.0, 0.0);
      A[f * Mp + padi(N)] = make_double2(0.0, 0.0);
    }
    if (a.rsrc) {
      // the coarse right-hand side from the fine residual (x pass: element
      // j of the line at tile coordinate u, remaining coordinate w is coarse
      // node (j, u, w)); one coarse value per thread and round, its 27 fine
      // loads in flight together
      for (int idx = threadIdx.x; idx < total; idx += KFBI_BLOCK) {
        int l, j;
        tile_pos(a, idx, nl, l, j);
        double xv = 0.0;
        if (u0 + l <= nl)
          xv = a.rsrc_f32 ? (double)restrict_fine<float>((const float*)a.rsrc, a.n1f, j, u0 + l, w)
                          : restrict_fine<double>((const double*)a.rsrc, a.n1f, j, u0 + l, w);
        double2* z = A + (l >> 1) * Mp;
        if (l & 1) {
          z[padi(j)].y = xv;
          z[padi(M - j)].y = -xv;
        } else {
          z[padi(j)].x = xv;
          z[padi(M - j)].x = -xv;
        }
      }
    } else
    // all loads of a chunk are issued before the LDS stores
    for (int base = threadIdx.x; base < total; base += DST_CH * KFBI_BLOCK) {
      double xv[DST_CH];
#pragma unroll
      for (int q = 0; q < DST_CH; ++q) {
        const int idx = base + q * KFBI_BLOCK;
        int l, j;
        tile_pos(a, idx, nl, l, j);
        xv[q] = (idx < total && u0 + l <= nl) ? a.in[elem_addr(a, u0 + l, w, j)] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < DST_CH; ++q) {
        const int idx = base + q * KFBI_BLOCK;
        if (idx >= total) continue;
        int l, j;
        tile_pos(a, idx, nl, l, j);
        double2* z = A + (l >> 1) * Mp;
        if (l & 1) {
          z[padi(j)].y = xv[q];
          z[padi(M - j)].y = -xv[q];
        } else {
          z[padi(j)].x = xv[q];
          z[padi(M - j)].x = -xv[q];
        }
      }
    }
  }
  __syncthreads();
  if (stop) return;
  if constexpr (FS) {
    // one sequence (nf = 1): the four-step FFT from the staged tile, the
    // sine coefficients stored straight from its registers
    const int th = threadIdx.x, n2 = th >> 2, c = th & 3;
    double2 v[4], y[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) v[m] = A[padi(64 * (c + 4 * m) + n2)];
    fft1024_regs(v, B, T4, y);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = fs_out_index(q);
      if (k < 1 || k > nl) continue;
      a.out[elem_addr(a, u0, w, k)] = -0.5 * y[q].y;
      if (u0 + 1 <= nl) a.out[elem_addr(a, u0 + 1, w, k)] = 0.5 * y[q].x;
    }
    return;
  }
  double2* R = fft_stockham<LOGM>(A, B, T, nf);
  if (MODE == 1) {
    // S_A(k) = -Im Z_k / 2 (even line), S_B(k) = Re Z_k / 2 (odd line); divide
    // by lambda, scale, and form the odd sequences of the inverse transform.
    // Lines past the grid (u > N-1) carry zeros and take s_u = s_1, a
    // nonzero lambda, so they stay zero.
    double2* S = R == A ? B : A;
    for (int f = threadIdx.x; f < nf; f += blockDim.x) {
      S[f * Mp] = make_double2(0.0, 0.0);
      S[f * Mp + padi(N)] = make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int k = threadIdx.x + q * KFBI_BLOCK;
      if (k < 1 || k > nl) continue;
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        if (f >= nf) break;
        const double2 Z = R[f * Mp + padi(k)];
        const double lamA = eigenvalue(g, sk[q], su[2 * f], sw);
        const double lamB = eigenvalue(g, sk[q], su[2 * f + 1], sw);
        const double2 c = make_double2(a.scale * (-0.5 * Z.y) / lamA, a.scale * (0.5 * Z.x) / lamB);
        S[f * Mp + padi(k)] = c;
        S[f * Mp + padi(M - k)] = make_double2(-c.x, -c.y);
      }
    }
    __syncthreads();
    R = fft_stockham<LOGM>(S, R, T, nf);
  }
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    int l, k;
    tile_pos(a, idx, nl, l, k);
    const int u = u0 + l;
    if (u > nl) continue;
    const double2 Z = R[(l >> 1) * Mp + padi(k)];
    a.out[elem_addr(a, u, w, k)] = (l & 1) ? 0.5 * Z.x : -0.5 * Z.y;
  }
}

// One axis pass over two lines of 511 interior nodes (N = 512, TL = 2,
// sequences of M = 1024) with the four-step FFT and no staging: each thread
// loads the four elements of the odd extension its first step needs
// straight from global memory (z[j] = (A_j, B_j), z[M - j] = -z[j], z[0] =
// z[N] = 0 for the tile's lines A and B), and stores the sine coefficients
// of the four outputs it ends with straight to global memory.  MODE 1
// divides those outputs by the eigenvalues, writes the odd extension of the
// divided spectrum to LDS and transforms it again.
template <int MODE>
__device__ __forceinline__ void dst1024_pass(const DstArgs& a, const int tile) {
  if (a.mctl && a.mctl[0]) return;
  const int stop = a.ctl ? a.ctl[1] : 0;
  constexpr int M = 1024, N = 512, nl = N - 1, Mp = padded_len(M);
  __shared__ double2 S[MODE == 1 ? Mp : 1];   // divided spectrum (MODE 1)
  __shared__ double2 X[Mp];                   // transpose buffer
  const GridDesc& g = a.g;
  const int w = tile / a.tiles_u + 1;
  const int u0 = 1 + (tile % a.tiles_u) * 2;
  const bool hasB = u0 + 1 <= nl;
  const int th = threadIdx.x, n2 = th >> 2, c = th & 3;
  Tw4 T;
  T.load(a.tw);
  double xa[4], xb[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int j = 64 * (c + 4 * m) + n2;
    const int jj = j < N ? j : M - j;
    const bool ok = jj >= 1 && jj <= nl;
    xa[m] = ok ? a.in[elem_addr(a, u0, w, jj)] : 0.0;
    xb[m] = ok && hasB ? a.in[elem_addr(a, u0 + 1, w, jj)] : 0.0;
  }
  int kk[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) kk[q] = fs_out_index(q);
  double sk[4], suA = 0.0, suB = 0.0, sw = 0.0;
  if (MODE == 1) {
#pragma unroll
    for (int q = 0; q < 4; ++q) sk[q] = (kk[q] >= 1 && kk[q] <= nl) ? a.eig1[kk[q]] : 0.0;
    suA = a.eig1[u0];
    suB = a.eig1[hasB ? u0 + 1 : 1];
    if (g.d == 3) sw = a.eig1[w];
  }
  if (stop) return;
  double2 v[4], y[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const bool lower = 64 * (c + 4 * m) + n2 < N;
    v[m] = lower ? make_double2(xa[m], xb[m]) : make_double2(-xa[m], -xb[m]);
  }
  fft1024_regs(v, X, T, y);
  if (MODE == 1) {
    // S_A(k) = -Im Z_k / 2, S_B(k) = Re Z_k / 2, divided by lambda and
    // scaled, as the odd sequence of the inverse transform
    if (th == 0) {
      S[padi(0)] = make_double2(0.0, 0.0);
      S[padi(N)] = make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = kk[q];
      if (k < 1 || k > nl) continue;
      const double lamA = eigenvalue(g, sk[q], suA, sw);
      const double lamB = eigenvalue(g, sk[q], suB, sw);
      const double2 cf = make_double2(a.scale * (-0.5 * y[q].y) / lamA, a.scale * (0.5 * y[q].x) / lamB);
      S[padi(k)] = cf;
      S[padi(M - k)] = make_double2(-cf.x, -cf.y);
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 4; ++m) v[m] = S[padi(64 * (c + 4 * m) + n2)];
    fft1024_regs(v, X, T, y);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int k = kk[q];
    if (k < 1 || k > nl) continue;
    a.out[elem_addr(a, u0, w, k)] = -0.5 * y[q].y;
    if (hasB) a.out[elem_addr(a, u0 + 1, w, k)] = 0.5 * y[q].x;
  }
}

// Tiles in XCD-contiguous order (neighbouring tiles share cache lines along
// the strided axes).
template <int LOGM, int MODE, bool FS>
__global__ void __launch_bounds__(KFBI_BLOCK) k_dst(DstArgs a) {
  dst_pass<LOGM, MODE, FS>(a, kfbi_xcd_block(blockIdx.x, gridDim.x));
}

template <int MODE>
__global__ void __launch_bounds__(KFBI_BLOCK) k_dst1024(DstArgs a) {
  dst1024_pass<MODE>(a, kfbi_xcd_block(blockIdx.x, gridDim.x));
}

// The same pass for several problems of one grid shape in one launch: work
// group b (in XCD-contiguous order over the whole launch) does tile b mod
// nbp of problem b / nbp, whose arguments it reads from A.
template <int LOGM, int MODE, bool FS>
__global__ void __launch_bounds__(KFBI_BLOCK) k_dstb(const DstArgs* __restrict__ A, int nbp) {
  const int lb = kfbi_xcd_block(blockIdx.x, gridDim.x);
  const DstArgs a = A[lb / nbp];
  dst_pass<LOGM, MODE, FS>(a, lb % nbp);
}

template <int MODE>
__global__ void __launch_bounds__(KFBI_BLOCK) k_dst1024b(const DstArgs* __restrict__ A, int nbp) {
  const int lb = kfbi_xcd_block(blockIdx.x, gridDim.x);
  const DstArgs a = A[lb / nbp];
  dst1024_pass<MODE>(a, lb % nbp);
}

// The same pass for problems of different grid sizes (N = 8..256, any
// mix) in one launch: start[p] is the first work group of problem p (its
// tiles follow in order); work group b (in XCD-contiguous order over the
// whole launch) finds its problem by bisection over start and runs that
// problem's pass body for its size, with that problem's arguments, so the
// arithmetic is the one of the problem's own launch.  The dynamic LDS is
// sized for the largest tile of the group.
template <int MODE>
__global__ void __launch_bounds__(KFBI_BLOCK) k_dstm(const DstArgs* __restrict__ A, const int* __restrict__ start,
                                                   int G) {
  const int lb = kfbi_xcd_block(blockIdx.x, gridDim.x);
  int lo = 0, hi = G;   // start[lo] <= lb < start[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= lb)
      lo = mid;
    else
      hi = mid;
  }
  const DstArgs a = A[lo];
  const int tile = lb - start[lo];
  switch (a.g.N) {
    case 8: dst_pass<4, MODE, false>(a, tile); break;
    case 16: dst_pass<5, MODE, false>(a, tile); break;
    case 32: dst_pass<6, MODE, false>(a, tile); break;
    case 64: dst_pass<7, MODE, false>(a, tile); break;
    case 128: dst_pass<8, MODE, false>(a, tile); break;
    default: dst_pass<9, MODE, false>(a, tile); break;
  }
}

// lines per tile, the built-in rule: the largest even TL <= 8 whose LDS
// footprint still lets 4 work groups (16 waves) share a compute unit and
// that leaves at least 1024 tiles (4 per compute unit); else 2.  More lines
// per tile amortise a work group's fixed latency; the residency and
// tile-count floors keep enough loads in flight.  (Measured on the 3D
// 64/128/256 and 2D grids: TL = 2, 8, 4 and 2 respectively.)
int tile_rule(int d, int N) {
  const int nl = N - 1;
  const int64_t lines = d == 3 ? (int64_t)nl * nl : nl;
  // 64^3 (the coarse grid of the 128^3 two-grid cycle): two 128-point
  // sequences per work group instead of one (993 tiles)
  if (d == 3 && N == 64) return 4;
  for (int tl = 8; tl > 2; tl -= 2) {
    if (tile_lds(tl, N) * 4 > DST_LDS_CU) continue;
    if ((lines + tl - 1) / tl < 1024) continue;
    return tl;
  }
  return 2;
}

// The tile lines in use per grid (dim, log2 N): a caller's override, else
// the autotuner's measurement, else the rule.  A line's transform does not
// depend on the tile it is in (lines are paired the same way for every even
// TL), so results are the same bit for bit whatever the choice.
std::atomic<int> g_tl_forced[2][12];
std::atomic<int> g_tl_tuned[2][12];
std::mutex g_tune_mu;

int log2i(int N) {
  int l = 0;
  while ((1 << l) < N) ++l;
  return l;
}

int tile_lines(int d, int N) {
  const int l = log2i(N);
  if (d >= 2 && d <= 3 && l < 12) {
    const int f = g_tl_forced[d - 2][l].load(std::memory_order_relaxed);
    if (f > 0) return f;
    const int t = g_tl_tuned[d - 2][l].load(std::memory_order_relaxed);
    if (t > 0) return t;
  }
  return tile_rule(d, N);
}

// the tile line counts worth trying for a grid: even, at most 8, at least
// two work groups' LDS per compute unit and 256 tiles (one per CU); the
// 2D grids of 512 and 1024 run their own kernels with fixed tiles
std::vector<int> tile_candidates(int d, int N) {
  std::vector<int> out;
  if (d == 2 && N >= 512) return out;
  const int64_t nl = N - 1, lines = d == 3 ? nl * nl : nl;
  for (int tl = 2; tl <= 8; tl += 2)
    if (tile_lds(tl, N) * 2 <= DST_LDS_CU && (lines + tl - 1) / tl >= 256) out.push_back(tl);
  return out;
}

template <int LOGM>
void launch_t(const DstArgs& a, unsigned blocks, size_t lds, hipStream_t st) {
  // one sequence of 1024 per work group (the corrected right-hand side's
  // pass; the others go to k_dst1024): the four-step FFT
  if constexpr (LOGM == 10) {
    if (a.TL == 2 && a.mode == 0 && KFBI_BLOCK == 256) {
      hipLaunchKernelGGL((k_dst<10, 0, true>), dim3(blocks), dim3(KFBI_BLOCK), lds, st, a);
      return;
    }
  }
  if (a.mode == 1)
    hipLaunchKernelGGL((k_dst<LOGM, 1, false>), dim3(blocks), dim3(KFBI_BLOCK), lds, st, a);
  else
    hipLaunchKernelGGL((k_dst<LOGM, 0, false>), dim3(blocks), dim3(KFBI_BLOCK), lds, st, a);
}

// launch one axis pass; a.g, a.ax, a.mode, a.in, a.out, a.tw, a.eig1 and
// the corrected-source fields are set by the caller
void launch_args(DstArgs& a, bool src_corr, hipStream_t st, int tl = 0) {
  const GridDesc& g = a.g;
  const int N = g.N, nl = N - 1;
  a.TL = tl > 0 ? tl : tile_lines(g.d, N);
  a.tiles_u = (nl + a.TL - 1) / a.TL;
  a.scale = 1.0;
  for (int t = 0; t < g.d; ++t) a.scale *= 2.0 / N;
  const unsigned blocks = (unsigned)(a.tiles_u * (g.d == 3 ? nl : 1));
  if (N == 512 && a.TL == 2 && !src_corr && KFBI_BLOCK == 256) {
    if (a.mode == 1)
      hipLaunchKernelGGL(k_dst1024<1>, dim3(blocks), dim3(KFBI_BLOCK), 0, st, a);
    else
      hipLaunchKernelGGL(k_dst1024<0>, dim3(blocks), dim3(KFBI_BLOCK), 0, st, a);
    return;
  }
  const size_t lds = tile_lds(a.TL, N);
  switch (N) {   // N is a power of two in [8, 1024]
    case 8: launch_t<4>(a, blocks, lds, st); break;
    case 16: launch_t<5>(a, blocks, lds, st); break;
    case 32: launch_t<6>(a, blocks, lds, st); break;
    case 64: launch_t<7>(a, blocks, lds, st); break;
    case 128: launch_t<8>(a, blocks, lds, st); break;
    case 256: launch_t<9>(a, blocks, lds, st); break;
    case 512: launch_t<10>(a, blocks, lds, st); break;
    default: launch_t<11>(a, blocks, lds, st); break;
  }
}

void launch_pass(kfbi_plan* pl, int ax, int mode, const double* in, double* out, bool src_corr = false) {
  DstArgs a{};
  a.ctl = pl->ctl_active;
  a.mctl = nullptr;
  a.src_corr = src_corr ? 1 : 0;
  a.row_start = pl->row_start;
  a.row_end = pl->row_end;
  a.irr = pl->irr;
  a.PE1 = pl->PE1;
  a.PE2 = pl->PE2;
  a.PA = pl->PA;
  a.Cv = pl->Cv;
  a.Firr = kfbi_irr_rhs_used(pl) ? pl->Firr : nullptr;
  a.maxpairs = pl->maxpairs;
  a.g = pl->g;
  a.ax = ax;
  a.mode = mode;
  a.in = in;
  a.out = out;
  a.tw = (const double2*)pl->tw;
  a.eig1 = pl->eig1;
  launch_args(a, src_corr, pl->stream);
}

// the arguments of pass q of the matvec's box solve of pl (as
// dst_solve_corrections launches them), with the plan's GMRES control word
DstArgs corrections_args(kfbi_plan* pl, int q) {
  static const int ax2[3] = {0, 1, 0}, md2[3] = {0, 1, 0};
  static const int ax3[5] = {0, 1, 2, 1, 0}, md3[5] = {0, 0, 1, 0, 0};
  DstArgs a{};
  a.ctl = pl->ctl;
  a.mctl = nullptr;
  a.src_corr = q == 0 ? 1 : 0;
  a.row_start = pl->row_start;
  a.row_end = pl->row_end;
  a.irr = pl->irr;
  a.PE1 = pl->PE1;
  a.PE2 = pl->PE2;
  a.PA = pl->PA;
  a.Cv = pl->Cv;
  a.Firr = kfbi_irr_rhs_used(pl) ? pl->Firr : nullptr;
  a.maxpairs = pl->maxpairs;
  a.g = pl->g;
  const bool d2 = pl->g.d == 2;
  a.ax = d2 ? ax2[q] : ax3[q];
  a.mode = d2 ? md2[q] : md3[q];
  double* const in2[3] = {nullptr, pl->T1, pl->T2};
  double* const out2[3] = {pl->T1, pl->T2, pl->vbuf};
  double* const in3[5] = {nullptr, pl->T1, pl->T2, pl->T1, pl->T2};
  double* const out3[5] = {pl->T1, pl->T2, pl->T1, pl->T2, pl->vbuf};
  a.in = d2 ? in2[q] : in3[q];
  a.out = d2 ? out2[q] : out3[q];
  a.tw = (const double2*)pl->tw;
  a.eig1 = pl->eig1;
  const int N = pl->g.N, nl = N - 1;
  a.TL = tile_lines(pl->g.d, N);
  a.tiles_u = (nl + a.TL - 1) / a.TL;
  a.scale = 1.0;
  for (int t = 0; t < pl->g.d; ++t) a.scale *= 2.0 / N;
  return a;
}

template <int LOGM>
void launch_tb(const DstArgs& a0, const DstArgs* A, int G, unsigned nbp, size_t lds, hipStream_t st) {
  const dim3 grid(nbp * (unsigned)G);
  if constexpr (LOGM == 10) {
    if (a0.TL == 2 && a0.mode == 0 && a0.src_corr && KFBI_BLOCK == 256) {
      hipLaunchKernelGGL((k_dstb<10, 0, true>), grid, dim3(KFBI_BLOCK), lds, st, A, (int)nbp);
      return;
    }
  }
  if (a0.mode == 1)
    hipLaunchKernelGGL((k_dstb<LOGM, 1, false>), grid, dim3(KFBI_BLOCK), lds, st, A, (int)nbp);
  else
    hipLaunchKernelGGL((k_dstb<LOGM, 0, false>), grid, dim3(KFBI_BLOCK), lds, st, A, (int)nbp);
}

// one pass of G problems of one shape: a0 the host copy of the first
// problem's arguments (shape, mode, tiles), A the G arguments on the device
void launch_batched(const DstArgs& a0, const DstArgs* A, int G, hipStream_t st) {
  const GridDesc& g = a0.g;
  const int N = g.N, nl = N - 1;
  const unsigned nbp = (unsigned)(a0.tiles_u * (g.d == 3 ? nl : 1));
  if (N == 512 && a0.TL == 2 && !a0.src_corr && KFBI_BLOCK == 256) {
    if (a0.mode == 1)
      hipLaunchKernelGGL(k_dst1024b<1>, dim3(nbp * (unsigned)G), dim3(KFBI_BLOCK), 0, st, A, (int)nbp);
    else
      hipLaunchKernelGGL(k_dst1024b<0>, dim3(nbp * (unsigned)G), dim3(KFBI_BLOCK), 0, st, A, (int)nbp);
    return;
  }
  const size_t lds = tile_lds(a0.TL, N);
  switch (N) {
    case 8: launch_tb<4>(a0, A, G, nbp, lds, st); break;
    case 16: launch_tb<5>(a0, A, G, nbp, lds, st); break;
    case 32: launch_tb<6>(a0, A, G, nbp, lds, st); break;
    case 64: launch_tb<7>(a0, A, G, nbp, lds, st); break;
    case 128: launch_tb<8>(a0, A, G, nbp, lds, st); break;
    case 256: launch_tb<9>(a0, A, G, nbp, lds, st); break;
    case 512: launch_tb<10>(a0, A, G, nbp, lds, st); break;
    default: launch_tb<11>(a0, A, G, nbp, lds, st); break;
  }
}

}  // namespace

// Batched matvec box solves of a group of plans of one dimension (FFT box
// solver): the arguments of every pass of every plan, on the device.  The
// plans with N <= 256 share one launch per pass (k_dstm); the larger ones,
// whose passes are other kernels (the register four-step FFT at N = 512),
// one launch per pass per grid size (k_dstb, k_dst1024b).
struct DstBatch {
  int npass = 0;
  int G = 0;                   // plans
  int Gm = 0;                  // plans in the mixed launch (the first Gm of the order below)
  size_t lds_m = 0;            // dynamic LDS of the mixed launch
  unsigned blocks_m = 0;       // work groups of the mixed launch
  std::vector<int> order;      // plan index of each slot: mixed ones, then the large ones by size
  std::vector<std::pair<int, int>> big;   // (first slot, count) per large grid size
  std::vector<DstArgs> host;   // [npass][G] in slot order
  DstArgs* dev = nullptr;      // [npass][G]
  int* start = nullptr;        // [Gm + 1] first work group of each mixed plan
};

DstBatch* dst_batch_create(kfbi_plan* const* pls, int G, hipStream_t st, kfbi_status* status) {
  *status = KFBI_OK;
  DstBatch* b = new (std::nothrow) DstBatch();
  if (!b) {
    *status = KFBI_E_OOM;
    return nullptr;
  }
  b->G = G;
  b->npass = pls[0]->g.d == 2 ? 3 : 5;
  for (int p = 0; p < G; ++p)
    if (pls[p]->g.N <= 256) b->order.push_back(p);
  b->Gm = (int)b->order.size();
  for (int N = 512; N <= 1024; N *= 2) {
    const int first = (int)b->order.size();
    for (int p = 0; p < G; ++p)
      if (pls[p]->g.N == N) b->order.push_back(p);
    if ((int)b->order.size() > first) b->big.push_back({first, (int)b->order.size() - first});
  }
  b->host.resize((size_t)b->npass * G);
  for (int q = 0; q < b->npass; ++q)
    for (int i = 0; i < G; ++i) b->host[(size_t)q * G + i] = corrections_args(pls[b->order[i]], q);
  std::vector<int> start(b->Gm + 1, 0);
  for (int i = 0; i < b->Gm; ++i) {
    const DstArgs& a = b->host[i];
    const int nl = a.g.N - 1;
    start[i + 1] = start[i] + a.tiles_u * (a.g.d == 3 ? nl : 1);
    const size_t l = tile_lds(a.TL, a.g.N);
    if (l > b->lds_m) b->lds_m = l;
  }
  b->blocks_m = (unsigned)start[b->Gm];
  if (hipMalloc((void**)&b->dev, sizeof(DstArgs) * b->host.size()) != hipSuccess ||
      hipMalloc((void**)&b->start, sizeof(int) * start.size()) != hipSuccess ||
      hipMemcpyAsync(b->dev, b->host.data(), sizeof(DstArgs) * b->host.size(), hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(b->start, start.data(), sizeof(int) * start.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    (void)hipGetLastError();
    kfbi_set_error("device allocation of the batched pass arguments failed");
    *status = KFBI_E_OOM;
    dst_batch_destroy(b);
    return nullptr;
  }
  return b;
}

void dst_batch_corrections(DstBatch* b, hipStream_t st) {
  for (int q = 0; q < b->npass; ++q) {
    const DstArgs* A = b->dev + (size_t)q * b->G;
    if (b->Gm > 0) {
      if (b->host[(size_t)q * b->G].mode == 1)
        hipLaunchKernelGGL(k_dstm<1>, dim3(b->blocks_m), dim3(KFBI_BLOCK), b->lds_m, st, A, b->start, b->Gm);
      else
        hipLaunchKernelGGL(k_dstm<0>, dim3(b->blocks_m), dim3(KFBI_BLOCK), b->lds_m, st, A, b->start, b->Gm);
    }
    for (const auto& g : b->big)
      launch_batched(b->host[(size_t)q * b->G + g.first], A + g.first, g.second, st);
  }
}

void dst_batch_destroy(DstBatch* b) {
  if (!b) return;
  if (b->dev) (void)hipFree(b->dev);
  if (b->start) (void)hipFree(b->start);
  delete b;
}

void dst_host_tables(int N, double h, double* tw, double* eig1) {
  const int M = 2 * N;
  for (int m = 0; m < M; ++m) {
    const double ang = -2.0 * M_PI * (double)m / (double)M;
    tw[2 * m] = cos(ang);
    tw[2 * m + 1] = sin(ang);
  }
  for (int k = 0; k <= N; ++k) {
    const double sn = sin((double)k * M_PI / (2.0 * N));
    eig1[k] = -4.0 / (h * h) * sn * sn;
  }
}

void dst_solve_grid(const GridDesc& g, const double* tw, const double* eig1, double* T1, double* T2,
                    const double* F, double* v, const int* ctl, const int* mctl, hipStream_t st,
                    const void* rsrc, int rsrc_f32, int n1f) {
  DstArgs a{};
  a.ctl = ctl;
  a.mctl = mctl;
  a.g = g;
  a.tw = (const double2*)tw;
  a.eig1 = eig1;
  // the passes of dst_solve: x, (y,) last axis with the divide, (y,) x
  const int n = g.d == 2 ? 3 : 5;
  const int ax2[3] = {0, 1, 0}, md2[3] = {0, 1, 0};
  const int ax3[5] = {0, 1, 2, 1, 0}, md3[5] = {0, 0, 1, 0, 0};
  const double* src[5] = {F, T1, T2, T1, T2};
  double* dst2[3] = {T1, T2, v};
  double* dst3[5] = {T1, T2, T1, T2, v};
  for (int q = 0; q < n; ++q) {
    a.ax = g.d == 2 ? ax2[q] : ax3[q];
    a.mode = g.d == 2 ? md2[q] : md3[q];
    a.in = src[q];
    a.out = g.d == 2 ? dst2[q] : dst3[q];
    // the first (x) pass forms the right-hand side from the fine residual
    a.rsrc = (q == 0 && g.d == 3) ? rsrc : nullptr;
    a.rsrc_f32 = rsrc_f32;
    a.n1f = n1f;
    launch_args(a, false, st);
  }
}

kfbi_status dst_init(kfbi_plan* pl) {
  int N = pl->g.N, M = 2 * N;
  std::vector<double> tw((size_t)2 * M), eig((size_t)N + 1);
  dst_host_tables(N, pl->g.h, tw.data(), eig.data());
  HIPCHK(hipMemcpyAsync(pl->tw, tw.data(), sizeof(double) * 2 * M, hipMemcpyHostToDevice, pl->stream));
  HIPCHK(hipMemcpyAsync(pl->eig1, eig.data(), sizeof(double) * (N + 1), hipMemcpyHostToDevice, pl->stream));
  HIPCHK(hipStreamSynchronize(pl->stream));
  const size_t lds = tile_lds(tile_lines(pl->g.d, N), N);
  if (N < 8 || N > 1024 || (N & (N - 1)) || lds > DST_LDS_CU) {
    kfbi_set_error("box solver LDS footprint too large (N = %d)", N);
    return KFBI_E_INVALID;
  }
  return dst_autotune_grid(pl->g, pl->tw, pl->eig1, pl->T1, pl->T2, pl->stream);
}

// Tile autotuner: at the first plan of a grid (dim, N) in the process (and
// at the first multigrid set-up for its coarse grid), time the x pass and
// the last (most strided) pass of the sine transform for every candidate
// tile (HIP events, three launches each after one warm-up, on that grid's
// own pass buffers) and keep the fastest for every later launch on that
// grid.  KFBI_TILE_AUTOTUNE=0 keeps the rule.
kfbi_status dst_autotune_grid(const GridDesc& g, const double* tw, const double* eig1, double* T1, double* T2,
                              hipStream_t st) {
  const int d = g.d, N = g.N, l = log2i(N);
  if (l >= 12 || g_tl_tuned[d - 2][l].load() > 0) return KFBI_OK;
  const char* env = getenv("KFBI_TILE_AUTOTUNE");
  if (env && env[0] == '0') return KFBI_OK;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (g_tl_tuned[d - 2][l].load() > 0) return KFBI_OK;
  const std::vector<int> cand = tile_candidates(d, N);
  const int rule = tile_rule(d, N);
  if (cand.size() < 2) {
    g_tl_tuned[d - 2][l].store(rule);
    return KFBI_OK;
  }
  HIPCHK(hipMemsetAsync(T1, 0, sizeof(double) * g.n_nodes, st));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return kfbi_hip_status(hipErrorOutOfMemory, "hipEventCreate");
  }
  int best = rule;
  float best_ms = -1.0f;
  kfbi_status status = KFBI_OK;
  for (int tl : cand) {
    float tot = 0.0f;
    for (int ax : {0, d - 1}) {
      DstArgs a{};
      a.g = g;
      a.ax = ax;
      a.mode = 0;
      a.in = T1;
      a.out = T2;
      a.tw = (const double2*)tw;
      a.eig1 = eig1;
      // one launch to warm up, then the faster of two rounds of eight
      launch_args(a, false, st, tl);
      float ms_min = -1.0f;
      for (int round = 0; round < 2 && status == KFBI_OK; ++round) {
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < 8; ++r) launch_args(a, false, st, tl);
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) {
          status = kfbi_hip_status(hipGetLastError(), "tile autotuner");
          break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms_min < 0.0f || ms < ms_min) ms_min = ms;
      }
      if (status != KFBI_OK) break;
      tot += ms_min;
    }
    if (status != KFBI_OK) break;
    // the rule's tile unless another is at least 10% faster (run-to-run
    // timing noise is a few percent; the choice should not flip with it)
    const bool better = best_ms < 0.0f || (tl == rule ? tot <= best_ms * 1.1f : tot * 1.1f < best_ms);
    if (better || (tl == rule && best != rule && tot <= best_ms * 1.1f)) {
      best = tl;
      best_ms = tot;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status == KFBI_OK) g_tl_tuned[d - 2][l].store(best);
  return status;
}

extern "C" int kfbi_tile_lines(int dim, int N) {
  if ((dim != 2 && dim != 3) || N < 8 || N > 1024 || (N & (N - 1))) return 0;
  return tile_lines(dim, N);
}

extern "C" kfbi_status kfbi_set_tile_lines(int dim, int N, int TL) {
  if ((dim != 2 && dim != 3) || N < 8 || N > 1024 || (N & (N - 1))) {
    kfbi_set_error("tile lines: dim 2 or 3 and N a power of two in [8, 1024]");
    return KFBI_E_INVALID;
  }
  const std::vector<int> cand = tile_candidates(dim, N);
  if (TL != 0 && std::find(cand.begin(), cand.end(), TL) == cand.end()) {
    kfbi_set_error("tile lines %d is not a candidate for dim %d, N %d", TL, dim, N);
    return KFBI_E_INVALID;
  }
  g_tl_forced[dim - 2][log2i(N)].store(TL);
  return KFBI_OK;
}

void dst_solve(kfbi_plan* pl, const double* F, double* v) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (pl->prof_on == 1 && pl->prof_ev && !pl->ctl_active) {
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
      (void)hipEventRecord(e0, pl->stream);
    } else {
      e0 = e1 = nullptr;
    }
  }
  if (pl->g.d == 2) {
    launch_pass(pl, 0, 0, F, pl->T1);
    launch_pass(pl, 1, 1, pl->T1, pl->T2);
    launch_pass(pl, 0, 0, pl->T2, v);
  } else {
    launch_pass(pl, 0, 0, F, pl->T1);
    launch_pass(pl, 1, 0, pl->T1, pl->T2);
    launch_pass(pl, 2, 1, pl->T2, pl->T1);
    launch_pass(pl, 1, 0, pl->T1, pl->T2);
    launch_pass(pl, 0, 0, pl->T2, v);
  }
  if (e0 && e1) {
    (void)hipEventRecord(e1, pl->stream);
    pl->prof_ev->push_back(e0);
    pl->prof_ev->push_back(e1);
    pl->prof_launches += pl->g.d == 2 ? 3 : 5;
  }
}

// box solve of the matvec: the right-hand side is formed from the density
// inside the first pass (no right-hand-side array)
void dst_solve_corrections(kfbi_plan* pl, const double* psi, double* v) {
  if (pl->g.d == 2) {
    launch_pass(pl, 0, 0, nullptr, pl->T1, true);
    launch_pass(pl, 1, 1, pl->T1, pl->T2);
    launch_pass(pl, 0, 0, pl->T2, v);
  } else {
    launch_pass(pl, 0, 0, nullptr, pl->T1, true);
    launch_pass(pl, 1, 0, pl->T1, pl->T2);
    launch_pass(pl, 2, 1, pl->T2, pl->T1);
    launch_pass(pl, 1, 0, pl->T1, pl->T2);
    launch_pass(pl, 0, 0, pl->T2, v);
  }
}

// ---------------------------------------------------------------- box solve without allocation
//
// kfbi_box_solve_noalloc: the FFT box solve of kfbi_box_solve (the same
// kernels) for a grid given by its parameters, with the two intermediate
// grids and the twiddle and eigenvalue tables in one file-scope device array
// instead of plan buffers, so a call allocates nothing.  Each device holds
// its own copy of the array until the process ends; its address on a device
// is looked up once (hipGetSymbolAddress) with that device current and kept.
namespace {

constexpr int NOALLOC_MAX_N2 = 1024;                   // 2D grids up to 1024^2
constexpr int NOALLOC_MAX_N3 = 128;                    // 3D grids up to 128^3
constexpr int64_t NOALLOC_GRID = 2146720;              // >= 129^3 and 1025^2, multiple of 32
constexpr int64_t NOALLOC_TW = 2 * 2 * NOALLOC_MAX_N2; // M = 2N complex twiddles
constexpr int64_t NOALLOC_EIG = 1280;                  // >= N + 1, multiple of 32
constexpr int64_t NOALLOC_DOUBLES = 2 * NOALLOC_GRID + NOALLOC_TW + NOALLOC_EIG;

__device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int NOALLOC_MAX_DEV = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_ptr[NOALLOC_MAX_DEV] = {};

// address of this device's scratch array (the symbol's name is a host-side
// stand-in, not a device address)
kfbi_status noalloc_scratch(double** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEV) {
    kfbi_set_error("device %d beyond the %d devices the static scratch table covers", dev, NOALLOC_MAX_DEV);
    return KFBI_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return kfbi_hip_status(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                      "hipGetSymbolAddress(scratch)");
    g_noalloc_ptr[dev] = (double*)p;
  }
  *out = g_noalloc_ptr[dev];
  return KFBI_OK;
}

// twiddles exp(-2 pi i m / 2N) and s_k = -4/h^2 sin^2(k pi / 2N), the tables
// dst_init writes from the host
__global__ void __launch_bounds__(KFBI_BLOCK) k_dst_tables(int N, double h, double* tw, double* eig1) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int M = 2 * N;
  if (i < M) {
    const double ang = -2.0 * M_PI * (double)i / (double)M;
    tw[2 * i] = cos(ang);
    tw[2 * i + 1] = sin(ang);
  }
  if (i <= N) {
    const double sn = sin((double)i * M_PI / (2.0 * N));
    eig1[i] = -4.0 / (h * h) * sn * sn;
  }
}

// zero box boundary of a grid array
__global__ void __launch_bounds__(KFBI_BLOCK) k_zero_box_boundary(GridDesc g, double* v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n_nodes) return;
  const int N = g.N;
  int64_t r = i;
  bool edge = false;
  for (int a = 0; a < g.d; ++a) {
    const int c = (int)(r % g.n1);
    r /= g.n1;
    edge = edge || c == 0 || c == N;
  }
  if (edge) v[i] = 0.0;
}

}  // namespace

extern "C" kfbi_status kfbi_box_solve_noalloc(int dim, int order, int N, double lo, double hi, double kappa,
                                              const double* F, double* v, void* stream) {
  if (dim != 2 && dim != 3) {
    kfbi_set_error("dim must be 2 or 3 (got %d)", dim);
    return KFBI_E_INVALID;
  }
  if (order != 2 && order != 4) {
    kfbi_set_error("order must be 2 or 4 (got %d)", order);
    return KFBI_E_INVALID;
  }
  const int nmax = dim == 2 ? NOALLOC_MAX_N2 : NOALLOC_MAX_N3;
  if (N < 8 || (N & (N - 1)) || N > nmax) {
    kfbi_set_error("N must be a power of two in [8, %d] for a %dD box solve without allocation (got %d): the "
                   "static scratch holds two grids of %lld values",
                   nmax, dim, N, (long long)NOALLOC_GRID);
    return KFBI_E_INVALID;
  }
  if (!(hi > lo) || !(kappa >= 0.0)) {
    kfbi_set_error("need hi > lo and kappa >= 0");
    return KFBI_E_INVALID;
  }
  if (!F || !v || F == v) {
    kfbi_set_error("box solve needs distinct F and v");
    return KFBI_E_INVALID;
  }
  GridDesc g{};
  g.d = dim;
  g.order = order;
  g.p = order == 4 ? 4 : 2;
  g.N = N;
  g.n1 = N + 1;
  g.K = 0;
  g.lo = lo;
  g.hi = hi;
  g.h = (hi - lo) / N;
  g.kappa = kappa;
  g.n_nodes = 1;
  for (int a = 0; a < dim; ++a) g.n_nodes *= g.n1;
  if (tile_lds(tile_lines(dim, N), N) > DST_LDS_CU) {
    kfbi_set_error("box solver LDS footprint too large (N = %d)", N);
    return KFBI_E_INVALID;
  }
  double* base = nullptr;
  KCHK(noalloc_scratch(&base));
  double* T1 = base;
  double* T2 = base + NOALLOC_GRID;
  double* tw = base + 2 * NOALLOC_GRID;
  double* eig1 = tw + NOALLOC_TW;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_dst_tables, dim3((2 * N + KFBI_BLOCK - 1) / KFBI_BLOCK), dim3(KFBI_BLOCK), 0, st, N, g.h, tw,
                     eig1);
  dst_solve_grid(g, tw, eig1, T1, T2, F, v, nullptr, nullptr, st);
  hipLaunchKernelGGL(k_zero_box_boundary, dim3((unsigned)((g.n_nodes + KFBI_BLOCK - 1) / KFBI_BLOCK)),
                     dim3(KFBI_BLOCK), 0, st, g, v);
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}
