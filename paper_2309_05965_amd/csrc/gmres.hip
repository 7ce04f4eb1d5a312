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

// r0 = b - A x0 (or b); beta = |r0|; V0 = r0 / beta; g0 = beta; scal[1] = |b|,
// scal[6] = beta (kept: scal[0] becomes the running residual estimate).
// Initialises the control word ctl = [j = 0, done, k = 0, max_iter] and the
// stopping threshold scal[3] = tol.
__global__ void __launch_bounds__(GB) k_start(int64_t n, const double* b, const double* Ax0, double* V,
                                             double* gv, double* scal, int* ctl, double tol, int maxit) {
  __shared__ double sh[GB];
  double sb = 0.0, sr = 0.0;
  // eight elements per thread per round, loads issued before the stores
  for (int64_t i0 = threadIdx.x; i0 < n; i0 += 8 * GB) {
    double bv[8], av[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t i = i0 + (int64_t)q * GB;
      bv[q] = i < n ? b[i] : 0.0;
      av[q] = (i < n && Ax0) ? Ax0[i] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t i = i0 + (int64_t)q * GB;
      if (i >= n) continue;
      const double r = Ax0 ? bv[q] - av[q] : bv[q];
      V[i] = r;
      sb += bv[q] * bv[q];
      sr += r * r;
    }
  }
  double nb = sqrt(block_sum(sb, sh));
  double beta = sqrt(block_sum(sr, sh));
  double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  for (int64_t i = threadIdx.x; i < n; i += GB) V[i] = V[i] * inv;
  if (threadIdx.x == 0) {
    gv[0] = beta;
    scal[0] = beta;
    scal[6] = beta;
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
// V[0..j] by classical Gram-Schmidt applied twice (CGS2), then normalised;
// the Givens rotations are applied to column j.  Every reduction runs in a
// fixed order, so the step is bitwise reproducible.
// DPP moves within a 16-lane row (register to register, no LDS): lane
// i ^ 1, i ^ 2 (quad permutes), i ^ 8 (row_ror:8), i ^ 7 (row_half_mirror)
template <int CTRL>
__device__ __forceinline__ double row_dpp(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)u, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
constexpr int RD_X1 = 0xB1, RD_X2 = 0x4E, RD_X3 = 0x1B, RD_X8 = 0x128, RD_X7 = 0x141;
__device__ __forceinline__ double row_x4(double v) { return row_dpp<RD_X3>(row_dpp<RD_X7>(v)); }   // lane i ^ 4

// eight sums over the 16 lanes of a row by a transposing butterfly of DPP
// moves: lanes 2k and 2k + 1 of the row end with the row's sum of p[k'],
// k' = row_reduce8_index(lane)
__device__ __forceinline__ double row_reduce8(const double (&p)[8], int lane) {
  const bool h8 = lane & 8, h4 = lane & 4, h2 = lane & 2;
  double a[4], b[2];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double send = h8 ? p[q] : p[q + 4];
    const double keep = h8 ? p[q + 4] : p[q];
    a[q] = keep + row_dpp<RD_X8>(send);
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const double send = h4 ? a[q] : a[q + 2];
    const double keep = h4 ? a[q + 2] : a[q];
    b[q] = keep + row_x4(send);
  }
  const double send = h2 ? b[0] : b[1];
  const double keep = h2 ? b[1] : b[0];
  const double c = keep + row_dpp<RD_X2>(send);
  return c + row_dpp<RD_X1>(c);
}

__device__ __forceinline__ int row_reduce8_index(int lane) {
  return ((lane & 8) ? 4 : 0) + ((lane & 4) ? 2 : 0) + ((lane & 2) ? 1 : 0);
}

// sum over the 16 lanes of a row (every lane of the row ends with it)
__device__ __forceinline__ double row_reduce(double v) {
  v += row_dpp<RD_X8>(v);
  v += row_x4(v);
  v += row_dpp<RD_X2>(v);
  return v + row_dpp<RD_X1>(v);
}

__device__ __forceinline__ double wave_reduce(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Givens rotations of Hessenberg column j held in hs[0..j+1] (hs[j+1] =
// |w|): the previous rotations (lcs, lsn) are applied in order, rotation j
// is formed and applied to g; the residual estimate |g_{j+1}|, the
// breakdown flag and the control word are updated.  One thread.
__device__ void givens_column(int j, double* hs, const double* lcs, const double* lsn, double* cs, double* sn,
                              double* gv, double* scal, int* ctl, bool breakdown) {
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

// Sum over the 64 lanes of eight per-lane values p[0..7] by a transposing
// butterfly: at xor distance 32, 16 and 8 each lane keeps half of its
// values and adds the partner's half, then three plain steps finish one
// value.  Lane l ends with the total of value 4 b5 + 2 b4 + b3 (b = bits of
// l); 10 shuffles instead of 48.  Fixed order, so reproducible.
__device__ __forceinline__ double wave_reduce8(const double (&p)[8], int lane) {
  const bool h32 = lane & 32, h16 = lane & 16, h8 = lane & 8;
  double a[4], b[2];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double send = h32 ? p[q] : p[q + 4];
    const double keep = h32 ? p[q + 4] : p[q];
    a[q] = keep + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const double send = h16 ? a[q] : a[q + 2];
    const double keep = h16 ? a[q + 2] : a[q];
    b[q] = keep + __shfl_xor(send, 16, 64);
  }
  double c;
  {
    const double send = h8 ? b[0] : b[1];
    const double keep = h8 ? b[1] : b[0];
    c = keep + __shfl_xor(send, 8, 64);
  }
  for (int off = 4; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  return c;
}

__device__ __forceinline__ int wave_reduce8_index(int lane) {
  return ((lane & 32) ? 4 : 0) + ((lane & 16) ? 2 : 0) + ((lane & 8) ? 1 : 0);
}

// Single work group (n <= 4096): w is staged in LDS for the whole step.
// (Beyond, one compute unit reading the whole basis takes longer than the
// four launches of the many-work-group chain.)
// A pass computes the j+1 dot products one wavefront per basis vector
// (lanes over the elements, eight loads of V in flight per lane, w from
// LDS, fixed-order wave reduction), then every thread updates its elements
// of w in LDS, eight basis vectors per round.
constexpr int ARN1_MAXN = 4096;
__global__ void __launch_bounds__(GB) k_arnoldi1(int64_t n, int* ctl, int ldh, double* V, double* Hm, double* cs,
                                                double* sn, double* gv, double* scal) {
  __shared__ double wl[ARN1_MAXN];
  __shared__ double hp[KFBI_GMRES_MAX + 1];
  __shared__ double hs[KFBI_GMRES_MAX + 2];
  __shared__ double lcs[KFBI_GMRES_MAX], lsn[KFBI_GMRES_MAX];
  __shared__ double red[GB / 64];
  if (ctl[1]) return;
  const int j = ctl[0];
  const int nn = (int)n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* w = V + (int64_t)(j + 1) * n;
  for (int t0 = threadIdx.x; t0 < nn; t0 += 8 * GB) {
    double x[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) x[q] = t0 + q * GB < nn ? w[t0 + q * GB] : 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (t0 + q * GB < nn) wl[t0 + q * GB] = x[q];
  }
  for (int i = threadIdx.x; i < j; i += GB) {
    lcs[i] = cs[i];
    lsn[i] = sn[i];
  }
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    for (int i = wave; i <= j; i += GB / 64) {
      const double* vi = V + (int64_t)i * n;
      double acc[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] = 0.0;
      for (int t0 = lane; t0 < nn; t0 += 8 * 64) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int t = t0 + 64 * q;
          if (t < nn) acc[q] += wl[t] * vi[t];
        }
      }
      const double sacc = wave_reduce(((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7])));
      if (lane == 0) hp[i] = sacc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= j; i += GB) hs[i] = pass == 0 ? hp[i] : hs[i] + hp[i];
    for (int t = threadIdx.x; t < nn; t += GB) {
      double v = wl[t];
      for (int i0 = 0; i0 <= j; i0 += 8) {
        double x[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) x[q] = i0 + q <= j ? V[(int64_t)(i0 + q) * n + t] : 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (i0 + q <= j) v -= hp[i0 + q] * x[q];
      }
      wl[t] = v;
    }
    __syncthreads();
  }
  double sq = 0.0;
  for (int t = threadIdx.x; t < nn; t += GB) sq += wl[t] * wl[t];
  sq = wave_reduce(sq);
  if (lane == 0) red[wave] = sq;
  __syncthreads();
  double tot = 0.0;
  for (int wv = 0; wv < GB / 64; ++wv) tot += red[wv];
  const double hn = sqrt(tot);
  const bool breakdown = !(hn > 0.0);
  const double inv = breakdown ? 1.0 : 1.0 / hn;
  for (int t = threadIdx.x; t < nn; t += GB) w[t] = breakdown ? wl[t] : wl[t] * inv;
  if (threadIdx.x == 0) {
    hs[j + 1] = hn;
    givens_column(j, hs, lcs, lsn, cs, sn, gv, scal, ctl, breakdown);
  }
  __syncthreads();
  double* hcol = Hm + (int64_t)j * ldh;
  for (int i = threadIdx.x; i <= j + 1; i += GB) hcol[i] = hs[i];
}

// value of x in lane l (l uniform across the wavefront)
__device__ __forceinline__ double lane_value(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Single work group, small n (n <= GB E): thread t holds elements t + GB r
// (r < E) of w and of the basis vectors V[0..JR-1] in registers for the
// whole step, so those are read from memory once, all loads in flight
// together; vectors JR..j (long runs) are read from memory when used.
// The coefficients are formed in chunks of 64 basis vectors: per-thread
// products, a sum of eight vectors at a time over the wavefront
// (transposing butterfly) into per-wavefront partials in LDS (two buffers
// used in turn, so one barrier per chunk), then every wavefront adds the
// NT / 64 partials of coefficient c0 + l in lane l and the update takes them from
// there (readlane).  Up to 64 basis vectors (every run seen in practice)
// this is exactly CGS2; beyond, each chunk is applied before the next
// one's coefficients are formed (block Gram-Schmidt over chunks).  The LDS
// footprint stays small (28 KB).
constexpr int ARN_CH = 64;

template <int E, int JR, int NT>
__global__ void __launch_bounds__(NT) k_arnoldi_reg(int64_t n, int* ctl, int ldh, double* V, double* Hm, double* cs,
                                                   double* sn, double* gv, double* scal) {
  static_assert(JR % 8 == 0 && JR <= ARN_CH, "register vectors: a multiple of 8, at most one chunk");
  // partials per row of 16 lanes (up to 512 threads) or per wavefront
  constexpr bool ROWS = NT <= 512;
  constexpr int NP = ROWS ? NT / 16 : NT / 64;
  __shared__ double red[2][NP][ARN_CH];
  __shared__ double hs[KFBI_GMRES_MAX + 2];
  __shared__ double lcs[KFBI_GMRES_MAX], lsn[KFBI_GMRES_MAX];
  __shared__ double rn[NP];
  if (ctl[1]) return;
  const int j = ctl[0];
  const int nn = (int)n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* w = V + (int64_t)(j + 1) * n;
  double wr[E], vr[JR][E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int t = threadIdx.x + NT * r;
    wr[r] = t < nn ? w[t] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < JR; ++i)
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int t = threadIdx.x + NT * r;
      vr[i][r] = (i <= j && t < nn) ? V[(int64_t)i * n + t] : 0.0;
    }
  for (int i = threadIdx.x; i < j; i += NT) {
    lcs[i] = cs[i];
    lsn[i] = sn[i];
  }
  int buf = 0;
  for (int pass = 0; pass < 2; ++pass) {
    for (int c0 = 0; c0 <= j; c0 += ARN_CH) {
      double(*rp)[ARN_CH] = red[buf];
      buf ^= 1;
      const int c1 = c0 + ARN_CH - 1 < j ? c0 + ARN_CH - 1 : j;   // last coefficient of the chunk
      if (c0 == 0) {
#pragma unroll
        for (int i0 = 0; i0 < JR; i0 += 8) {
          if (i0 > j) break;
          double p[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            double acc = 0.0;
#pragma unroll
            for (int r = 0; r < E; ++r) acc += vr[i0 + q][r] * wr[r];
            p[q] = acc;
          }
          if (ROWS) {
            const double sv = row_reduce8(p, lane);
            if ((lane & 1) == 0) rp[4 * wave + (lane >> 4)][i0 + row_reduce8_index(lane)] = sv;
          } else {
            const double sv = wave_reduce8(p, lane);
            if ((lane & 7) == 0) rp[wave][i0 + wave_reduce8_index(lane)] = sv;
          }
        }
      }
      for (int i0 = c0 == 0 ? JR : c0; i0 <= c1; i0 += 8) {
        double p[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          double acc = 0.0;
#pragma unroll
          for (int r = 0; r < E; ++r) {
            const int t = threadIdx.x + NT * r;
            if (i0 + q <= c1 && t < nn) acc += V[(int64_t)(i0 + q) * n + t] * wr[r];
          }
          p[q] = acc;
        }
        if (ROWS) {
          const double sv = row_reduce8(p, lane);
          if ((lane & 1) == 0 && i0 + row_reduce8_index(lane) <= c1)
            rp[4 * wave + (lane >> 4)][i0 - c0 + row_reduce8_index(lane)] = sv;
        } else {
          const double sv = wave_reduce8(p, lane);
          if ((lane & 7) == 0 && i0 + wave_reduce8_index(lane) <= c1) rp[wave][i0 - c0 + wave_reduce8_index(lane)] = sv;
        }
      }
      __syncthreads();
      double h0 = 0.0;                 // lane l: coefficient c0 + l of this pass
      if (c0 + lane <= c1)
        for (int wv = 0; wv < NP; ++wv) h0 += rp[wv][lane];
      if (wave == 0 && c0 + lane <= c1) hs[c0 + lane] = pass == 0 ? h0 : hs[c0 + lane] + h0;
      if (c0 == 0) {
#pragma unroll
        for (int r = 0; r < E; ++r) {
          double x = wr[r];
#pragma unroll
          for (int i = 0; i < JR; ++i)
            if (i <= j) x -= lane_value(h0, i) * vr[i][r];
          wr[r] = x;
        }
      }
      for (int i0 = c0 == 0 ? JR : c0; i0 <= c1; i0 += 8) {
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const int t = threadIdx.x + NT * r;
          double y[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) y[q] = (i0 + q <= c1 && t < nn) ? V[(int64_t)(i0 + q) * n + t] : 0.0;
          double x = wr[r];
#pragma unroll
          for (int q = 0; q < 8; ++q)
            if (i0 + q <= c1) x -= lane_value(h0, i0 + q - c0) * y[q];
          wr[r] = x;
        }
      }
    }
  }
  double sq = 0.0;
#pragma unroll
  for (int r = 0; r < E; ++r) sq += wr[r] * wr[r];
  if (ROWS) {
    sq = row_reduce(sq);
    if ((lane & 15) == 0) rn[4 * wave + (lane >> 4)] = sq;
  } else {
    sq = wave_reduce(sq);
    if (lane == 0) rn[wave] = sq;
  }
  __syncthreads();
  double tot = 0.0;
  for (int wv = 0; wv < NP; ++wv) tot += rn[wv];
  const double hn = sqrt(tot);
  const bool breakdown = !(hn > 0.0);
  const double inv = breakdown ? 1.0 : 1.0 / hn;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int t = threadIdx.x + NT * r;
    if (t < nn) w[t] = breakdown ? wr[r] : wr[r] * inv;
  }
  if (wave == 0) {
    if (lane == 0) {
      hs[j + 1] = hn;
      givens_column(j, hs, lcs, lsn, cs, sn, gv, scal, ctl, breakdown);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    double* hcol = Hm + (int64_t)j * ldh;
    for (int i = lane; i <= j + 1; i += 64) hcol[i] = hs[i];
  }
}

// Many work groups (large n): work group b owns w[b*AC .. b*AC + AC), AE
// elements per thread, and a step is four kernels.  Partial sums go to
// part[3][B][L] (L = gm_cap + 2); each consumer reduces them over b in a
// fixed order.  The first kernel copies (j, done) into ctl[4..5] for the
// last one, whose work group 0 advances ctl[0..3].
constexpr int AB = 256;          // threads per work group
constexpr int AE = 2;            // elements per thread
constexpr int AC = AB * AE;      // elements per work group

__device__ __forceinline__ int64_t arn_elem(int r) {
  return (int64_t)blockIdx.x * AC + threadIdx.x + (int64_t)AB * r;
}

// partial dot products of the work group's w (registers) with V[0..j] into
// out[0..j]
__device__ void arn_partial_dots(int64_t n, int j, const double* V, const double (&wr)[AE], double* out) {
  __shared__ double red[AB / 64][16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i0 = 0; i0 <= j; i0 += 16) {
    double p[2][8];
#pragma unroll
    for (int q = 0; q < 16; ++q) p[q >> 3][q & 7] = 0.0;
#pragma unroll
    for (int r = 0; r < AE; ++r) {
      const int64_t t = arn_elem(r);
      if (t < n) {
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if (i0 + q <= j) p[q >> 3][q & 7] += wr[r] * V[(int64_t)(i0 + q) * n + t];
      }
    }
#pragma unroll
    for (int hq = 0; hq < 2; ++hq) {
      const double sq = wave_reduce8(p[hq], lane);
      if ((lane & 7) == 0) red[wave][8 * hq + wave_reduce8_index(lane)] = sq;
    }
    __syncthreads();
    if (threadIdx.x < 16 && i0 + (int)threadIdx.x <= j)
      out[i0 + threadIdx.x] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
    __syncthreads();
  }
}

// h[i] = sum over b of part[b*L + i], i <= j, into LDS.  Thread t takes i =
// i0 + t mod 32 and every eighth b from t / 32, so the loads of all b are
// in flight together; the eight group sums are then added in order.
__device__ void arn_reduce(int j, int B, int L, const double* part, double* h) {
  __shared__ double tmp[8][32];
  const int ii = threadIdx.x & 31, g = threadIdx.x >> 5;
  for (int i0 = 0; i0 <= j; i0 += 32) {
    const int i = i0 + ii;
    double s = 0.0;
    if (i <= j)
      for (int b = g; b < B; b += 8) s += part[(int64_t)b * L + i];
    tmp[g][ii] = s;
    __syncthreads();
    if (threadIdx.x < 32 && i <= j) {
      double t = 0.0;
      for (int q = 0; q < 8; ++q) t += tmp[q][ii];
      h[i] = t;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(AB) k_arn_dots(int64_t n, int* ctl, const double* V, double* part, int L) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl[4] = ctl[0];
    ctl[5] = ctl[1];
  }
  if (ctl[1]) return;
  const int j = ctl[0];
  const double* w = V + (int64_t)(j + 1) * n;
  double wr[AE];
#pragma unroll
  for (int r = 0; r < AE; ++r) {
    const int64_t t = arn_elem(r);
    wr[r] = t < n ? w[t] : 0.0;
  }
  arn_partial_dots(n, j, V, wr, part + (int64_t)blockIdx.x * L);
}

// PASS 0: w -= V h1, then the partial dots of the new w (second pass);
// PASS 1: w -= V h2, then the partial sum of w^2
template <int PASS>
__global__ void __launch_bounds__(AB) k_arn_update(int64_t n, const int* ctl, double* V, const double* pin,
                                                  double* pout, int L, int B) {
  __shared__ double h[KFBI_GMRES_MAX + 1];
  __shared__ double red[AB / 64];
  if (ctl[1]) return;
  const int j = ctl[0];
  double* w = V + (int64_t)(j + 1) * n;
  double wr[AE];
#pragma unroll
  for (int r = 0; r < AE; ++r) {
    const int64_t t = arn_elem(r);
    wr[r] = t < n ? w[t] : 0.0;
  }
  arn_reduce(j, B, L, pin, h);
  for (int i0 = 0; i0 <= j; i0 += 8) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (i0 + q > j) break;
      const double hq = h[i0 + q];
#pragma unroll
      for (int r = 0; r < AE; ++r) {
        const int64_t t = arn_elem(r);
        if (t < n) wr[r] -= hq * V[(int64_t)(i0 + q) * n + t];
      }
    }
  }
#pragma unroll
  for (int r = 0; r < AE; ++r) {
    const int64_t t = arn_elem(r);
    if (t < n) w[t] = wr[r];
  }
  if (PASS == 0) {
    arn_partial_dots(n, j, V, wr, pout + (int64_t)blockIdx.x * L);
  } else {
    double sq = 0.0;
#pragma unroll
    for (int r = 0; r < AE; ++r) sq += wr[r] * wr[r];
    sq = wave_reduce(sq);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) pout[(int64_t)blockIdx.x * L] = ((red[0] + red[1]) + red[2]) + red[3];
  }
}

// |w| from the partial sums, w /= |w|; work group 0 forms the Hessenberg
// column h1 + h2, |w| and applies the Givens rotations
__global__ void __launch_bounds__(AB) k_arn_finish(int64_t n, int* ctl, int ldh, double* V, double* Hm, double* cs,
                                                  double* sn, double* gv, double* scal, const double* part, int L,
                                                  int B, int PB) {
  __shared__ double hs[KFBI_GMRES_MAX + 2];
  __shared__ double h2[KFBI_GMRES_MAX + 1];
  __shared__ double lcs[KFBI_GMRES_MAX], lsn[KFBI_GMRES_MAX];
  if (ctl[5]) return;
  const int j = ctl[4];
  __shared__ double nrm[1];
  arn_reduce(0, B, L, part + (int64_t)2 * PB * L, nrm);
  const double hn = sqrt(nrm[0]);
  const bool breakdown = !(hn > 0.0);
  const double inv = breakdown ? 1.0 : 1.0 / hn;
  double* w = V + (int64_t)(j + 1) * n;
#pragma unroll
  for (int r = 0; r < AE; ++r) {
    const int64_t t = arn_elem(r);
    if (t < n && !breakdown) w[t] = w[t] * inv;
  }
  if (blockIdx.x != 0) return;
  arn_reduce(j, B, L, part, hs);
  arn_reduce(j, B, L, part + (int64_t)PB * L, h2);
  for (int i = threadIdx.x; i <= j; i += AB) hs[i] += h2[i];
  for (int i = threadIdx.x; i < j; i += AB) {
    lcs[i] = cs[i];
    lsn[i] = sn[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    hs[j + 1] = hn;
    givens_column(j, hs, lcs, lsn, cs, sn, gv, scal, ctl, breakdown);
  }
  __syncthreads();
  double* hcol = Hm + (int64_t)j * ldh;
  for (int i = threadIdx.x; i <= j + 1; i += AB) hcol[i] = hs[i];
}

// y = H^{-1} g (upper triangular, k x k), then x = x0 + V^T y.  The
// triangle is staged in LDS (k <= 64) so the sequential back substitution
// reads no global memory.
// kdev non-null: the iteration count is read from the device (the
// GMRES control word), so the update can be enqueued before the host knows it
__global__ void __launch_bounds__(256) k_trisolve(int k, const int* kdev, int ldh, const double* Hm, const double* gv,
                                                 double* y) {
  __shared__ double H[64][65];
  __shared__ double gl[64];
  if (kdev) k = *kdev;
  if (k <= 0) return;
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

__global__ void k_combine(int64_t n, int k, const int* kdev, const double* V, const double* y, double* x, int use_x0) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (kdev) k = *kdev;
  double s = use_x0 ? x[i] : 0.0;
  for (int m = 0; m < k; ++m) s += V[(int64_t)m * n + i] * y[m];
  x[i] = s;
}

__global__ void __launch_bounds__(GB) k_resid(int64_t n, const double* b, const double* Ax, double* out) {
  __shared__ double sh[GB];
  double sr = 0.0, sb = 0.0;
  for (int64_t i0 = threadIdx.x; i0 < n; i0 += 8 * GB) {
    double bv[8], av[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t i = i0 + (int64_t)q * GB;
      bv[q] = i < n ? b[i] : 0.0;
      av[q] = i < n ? Ax[i] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double r = bv[q] - av[q];
      sr += r * r;
      sb += bv[q] * bv[q];
    }
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

// one work group up to 4096 unknowns (the step is latency-bound there),
// with the basis in registers up to 2048; beyond, the basis is read by many
// compute units
void gm_arnoldi(kfbi_plan* pl) {
  const int64_t n = pl->n_dof;
  const int ldh = pl->gm_cap + 1;
  hipStream_t st = pl->stream;
  // the fewest wavefronts whose registers hold the thread's elements of w
  // and of the first basis vectors: the step is bound by its cross-wave
  // reductions and barriers, which shrink with the wavefront count
  if (n <= 256) {
    hipLaunchKernelGGL((k_arnoldi_reg<1, 32, 256>), dim3(1), dim3(256), 0, st, n, pl->ctl, ldh, pl->V, pl->Hm,
                       pl->cs, pl->sn, pl->gv, pl->scal);
  } else if (n <= 512) {
    hipLaunchKernelGGL((k_arnoldi_reg<2, 32, 256>), dim3(1), dim3(256), 0, st, n, pl->ctl, ldh, pl->V, pl->Hm,
                       pl->cs, pl->sn, pl->gv, pl->scal);
  } else if (n <= GB) {
    hipLaunchKernelGGL((k_arnoldi_reg<2, 32, 512>), dim3(1), dim3(512), 0, st, n, pl->ctl, ldh, pl->V, pl->Hm,
                       pl->cs, pl->sn, pl->gv, pl->scal);
  } else if (n <= 5 * 256) {
    hipLaunchKernelGGL((k_arnoldi_reg<5, 16, 256>), dim3(1), dim3(256), 0, st, n, pl->ctl, ldh, pl->V, pl->Hm,
                       pl->cs, pl->sn, pl->gv, pl->scal);
  } else if (n <= 2 * GB) {
    hipLaunchKernelGGL((k_arnoldi_reg<2, 16, GB>), dim3(1), dim3(GB), 0, st, n, pl->ctl, ldh, pl->V, pl->Hm, pl->cs,
                       pl->sn, pl->gv, pl->scal);
  } else if (n <= ARN1_MAXN) {
    hipLaunchKernelGGL(k_arnoldi1, dim3(1), dim3(GB), 0, st, n, pl->ctl, ldh, pl->V, pl->Hm, pl->cs, pl->sn,
                       pl->gv, pl->scal);
  } else {
    const int B = (int)((n + AC - 1) / AC), L = pl->gm_cap + 2, PB = pl->gm_pb;
    double* p1 = pl->gm_part;
    double* p2 = p1 + (int64_t)PB * L;
    double* p3 = p2 + (int64_t)PB * L;
    hipLaunchKernelGGL(k_arn_dots, dim3(B), dim3(AB), 0, st, n, pl->ctl, pl->V, p1, L);
    hipLaunchKernelGGL(k_arn_update<0>, dim3(B), dim3(AB), 0, st, n, pl->ctl, pl->V, p1, p2, L, B);
    hipLaunchKernelGGL(k_arn_update<1>, dim3(B), dim3(AB), 0, st, n, pl->ctl, pl->V, p2, p3, L, B);
    hipLaunchKernelGGL(k_arn_finish, dim3(B), dim3(AB), 0, st, n, pl->ctl, ldh, pl->V, pl->Hm, pl->cs, pl->sn,
                       pl->gv, pl->scal, pl->gm_part, L, B, PB);
  }
}

int gm_part_blocks(int64_t n) { return (int)((n + AC - 1) / AC); }

void gm_update(kfbi_plan* pl, int k, double* x, int use_x0) {
  if (k > 0) hipLaunchKernelGGL(k_trisolve, dim3(1), dim3(256), 0, pl->stream, k, nullptr, pl->gm_cap + 1, pl->Hm,
                                pl->gv, pl->scal + 8);
  unsigned nbk = (unsigned)((pl->n_dof + KFBI_BLOCK - 1) / KFBI_BLOCK);
  hipLaunchKernelGGL(k_combine, dim3(nbk), dim3(KFBI_BLOCK), 0, pl->stream, pl->n_dof, k, nullptr, pl->V,
                     pl->scal + 8, x, use_x0);
}

// the same with the iteration count taken from the device control word
void gm_update_device(kfbi_plan* pl, double* x, int use_x0) {
  hipLaunchKernelGGL(k_trisolve, dim3(1), dim3(256), 0, pl->stream, 0, pl->ctl + 2, pl->gm_cap + 1, pl->Hm, pl->gv,
                     pl->scal + 8);
  unsigned nbk = (unsigned)((pl->n_dof + KFBI_BLOCK - 1) / KFBI_BLOCK);
  hipLaunchKernelGGL(k_combine, dim3(nbk), dim3(KFBI_BLOCK), 0, pl->stream, pl->n_dof, 0, pl->ctl + 2, pl->V,
                     pl->scal + 8, x, use_x0);
}

void gm_true_residual(kfbi_plan* pl, const double* b, const double* Ax, double* out2) {
  hipLaunchKernelGGL(k_resid, dim3(1), dim3(GB), 0, pl->stream, pl->n_dof, b, Ax, out2);
}
