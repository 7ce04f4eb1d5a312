// Step S3 / S8 -- multigrid box solver: two-grid cycles in FP32 (or FP64)
// inside an FP64 defect-correction loop.
//
// The box solve of Alg. 1 Step 3.3 is A_h v = F on the interior nodes with
// v = 0 on the box boundary.  The paper uses the FFT; this module is the
// multigrid alternative for the same system:
//   grids        the fine grid N and the coarse grid N/2, the compact operator
//                rediscretised with 2h (same reduced kappa);
//   smoother     damped Jacobi u <- u + (omega / a)(f - A u), a the central
//                coefficient, omega = 2 / (rho_lo + rho_hi) over the
//                high-frequency range of the symbol lambda(theta) / a;
//   transfers    full weighting (1/4, 1/2, 1/4)^d and (bi/tri)linear
//                interpolation;
//   coarse       solved exactly in FP64 by the sine transform (the passes of
//                the FFT box solver on the coarse grid);
//   cycle        two pre- and two post-smoothing steps from a zero guess.
// Defect correction: r = F - A_h v in FP64, then one cycle on (T) r in the
// inner precision T, v <- v + e, until |r|_2 <= eps |F|_2 or max_cycles
// corrections.  All grids carry their boundary (zero) so every stencil
// access is in bounds without branches.  Every kernel reads a device control
// word and returns at once when the loop has converged, so the whole
// schedule can be captured in a graph; it also honours the GMRES control
// word when it runs inside a captured GMRES iteration.
//
// Design for gfx950: at 128^3 the kernels of the lower levels of a deep
// V-cycle (64^3, 32^3 and an in-LDS cycle below) cost about as much as the
// fine level, every one of them latency-bound; the exact coarse solve
// replaces all of them by five sine-transform passes and converges faster
// per cycle (0.07 against 0.09 on the fourth-order operators).
#include <math.h>

#include <vector>

#include <string.h>

#include "kfbi_internal.h"

namespace {

constexpr int MG_BLOCK = 256;
constexpr int MG_PART = 8192;            // partial sums of the outer residual (per block)
constexpr int CHECK_BLOCK = 1024;        // threads of the stopping test

template <typename T>
struct Lev {
  int N, n1, d;
  int64_t off;       // element offset of this level in the level arrays
  T c[27];           // A_l on the 3^d cube, index (o0+1) + 3 (o1+1) + 9 (o2+1)
  T coef;            // omega_l / a_l
  T inva;            // 1 / a_l
  int star;          // only the centre and axis neighbours are nonzero (2nd order)
};

// sum of c[q] val(o) over the 3^D cube (index q = (o0+1) + 3 (o1+1) + 9 (o2+1),
// 2D on the o2 = 0 plane) in the order of q; with star only the centre and
// axis terms, which are the nonzero ones then.  No data-dependent branch:
// a skipped zero coefficient adds +0, so the full form equals the sum
// over the nonzero terms for finite values.
template <int D, typename S, typename F>
__device__ __forceinline__ S stencil_sum(const S* c, bool star, F val) {
  S s = 0;
  if (star) {
#pragma unroll
    for (int q = 0; q < 27; ++q) {
      const int o0 = q % 3 - 1, o1 = (q / 3) % 3 - 1, o2 = q / 9 - 1;
      if (D == 2 && o2 != 0) continue;
      if ((o0 != 0) + (o1 != 0) + (o2 != 0) > 1) continue;
      s += c[q] * val(o0, o1, o2);
    }
  } else {
#pragma unroll
    for (int q = 0; q < 27; ++q) {
      const int o0 = q % 3 - 1, o1 = (q / 3) % 3 - 1, o2 = q / 9 - 1;
      if (D == 2 && o2 != 0) continue;
      s += c[q] * val(o0, o1, o2);
    }
  }
  return s;
}

// star test of a 27-entry stencil (host)
inline int stencil_is_star(const double* c) {
  for (int q = 0; q < 27; ++q) {
    const int o0 = q % 3 - 1, o1 = (q / 3) % 3 - 1, o2 = q / 9 - 1;
    if ((o0 != 0) + (o1 != 0) + (o2 != 0) > 1 && c[q] != 0.0) return 0;
  }
  return 1;
}

struct Ctl {
  const int* gctl;   // GMRES control word (captured iteration) or null
  int* mctl;         // [done, corrections done]
};

__device__ __forceinline__ bool skip(const Ctl& c) { return (c.gctl && c.gctl[1]) || c.mctl[0]; }

// sums of a and b over the work group (NT threads): a butterfly within each
// wavefront, then the wavefront sums in order (one barrier); the results
// are valid in thread 0.  sh holds 2 NT / 64 values.
template <int NT>
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
  }
  constexpr int NW = NT / 64;
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[w] = a;
    sh[NW + w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = sh[0];
    b = sh[NW];
#pragma unroll
    for (int i = 1; i < NW; ++i) {
      a += sh[i];
      b += sh[NW + i];
    }
  }
}

// grid index of interior node t (x fastest); grids have at most 1025^3
// nodes, so 32-bit arithmetic is exact
__device__ __forceinline__ int64_t node_of(int d, int n1, int64_t t64, int N) {
  const unsigned m = (unsigned)(N - 1);
  const unsigned t = (unsigned)t64;
  const unsigned r = t / m;
  const unsigned i = t - r * m + 1;
  if (d == 2) return (int64_t)(i + (unsigned)n1 * (r + 1));
  const unsigned k = r / m;
  const unsigned j = r - k * m + 1;
  return (int64_t)(i + (unsigned)n1 * (j + (unsigned)n1 * (k + 1)));
}

// coordinates (i, j, k) of interior node t (32-bit arithmetic, as node_of)
__device__ __forceinline__ void node_ijk(int d, int64_t t64, int N, int& i, int& j, int& k) {
  const unsigned m = (unsigned)(N - 1);
  const unsigned t = (unsigned)t64;
  const unsigned r = t / m;
  i = (int)(t - r * m + 1);
  if (d == 2) {
    j = (int)(r + 1);
    k = 0;
    return;
  }
  const unsigned q = r / m;
  j = (int)(r - q * m + 1);
  k = (int)(q + 1);
}

// coarse value at coarse interior node I from the fine residual r
template <typename T>
__device__ __forceinline__ T op_restrict(int d, int n1f, const T* r, int I0, int I1, int I2) {
  const T w1[3] = {(T)0.25, (T)0.5, (T)0.25};
  const int zr = d == 3 ? 1 : 0;
  T s = 0;
  for (int o2 = -zr; o2 <= zr; ++o2)
    for (int o1 = -1; o1 <= 1; ++o1)
      for (int o0 = -1; o0 <= 1; ++o0) {
        T w = w1[o0 + 1] * w1[o1 + 1];
        if (d == 3) w *= w1[o2 + 1];
        const int64_t fi = (2 * I0 + o0) + (int64_t)n1f * ((2 * I1 + o1) + (int64_t)n1f * (d == 3 ? 2 * I2 + o2 : 0));
        s += w * r[fi];
      }
  return s;
}

// (bi/tri)linear interpolation of the coarse grid at fine node (i0,i1,i2)
template <typename T>
__device__ __forceinline__ T op_prolong(int d, int n1c, const T* e, int i0, int i1, int i2) {
  const int p0 = i0 & 1, p1 = i1 & 1, p2 = d == 3 ? (i2 & 1) : 0;
  const int I0 = i0 >> 1, I1 = i1 >> 1, I2 = d == 3 ? (i2 >> 1) : 0;
  T s = 0;
  for (int c2 = 0; c2 <= p2; ++c2)
    for (int c1 = 0; c1 <= p1; ++c1)
      for (int c0 = 0; c0 <= p0; ++c0) s += e[(I0 + c0) + (int64_t)n1c * ((I1 + c1) + (int64_t)n1c * (I2 + c2))];
  // the average of 2^(p0+p1+p2) values: the reciprocal is exact
  return s * ((T)1 / (T)(1 << (p0 + p1 + p2)));
}

__device__ __forceinline__ void coords(int d, int n1, int64_t idx, int& i0, int& i1, int& i2) {
  i0 = (int)(idx % n1);
  int64_t r = idx / n1;
  if (d == 2) {
    i1 = (int)r;
    i2 = 0;
  } else {
    i1 = (int)(r % n1);
    i2 = (int)(r / n1);
  }
}

// ---------------------------------------------------------------- global kernels
// Stencil sweeps of the fine levels.  A workgroup owns a tile of the plane
// transverse to the marching axis (3D: 64 x 4 nodes in x-y, marching along
// z; 2D: 256 nodes along x, marching along y) and a chunk of KZ planes; the
// planes z-1, z, z+1 of the stencil input (with a one-node halo) rotate
// through LDS, so every input value is read from memory about once.
enum { SW_SMOOTH = 0, SW_SMOOTH2 = 1, SW_RESID = 2, SW_OUTER = 3, SW_SMOOTH_UPD = 4, SW_PSMOOTH = 5 };

template <typename TS, typename TO>
struct SweepArgs {
  int N, n1, KZ;
  TS c[27];
  TS coef;           // omega / a
  int star;          // only centre and axis coefficients nonzero
  const TS* s;       // stencil input (u, or f for SW_SMOOTH2, or v for SW_OUTER)
  const TS* f;       // right-hand side (F for SW_OUTER)
  TO* out;
  double* part;      // SW_OUTER: per-block sums of r^2 (and F^2 at part + MG_PART)
  double* v;         // SW_SMOOTH_UPD: v += (double) smoothed value (out unused)
  int* mctl;         // SW_SMOOTH_UPD: corrections counter mctl[1], raised once
  const double* ec;  // SW_PSMOOTH: FP64 coarse correction (full coarse grid)
  int Nc, n1c;       // SW_PSMOOTH: coarse grid size
};

template <int D>
struct Tile {
  static constexpr int TX = D == 3 ? 64 : 256;
  static constexpr int TY = D == 3 ? 4 : 1;
  static constexpr int PX = TX + 2;
  static constexpr int PY = D == 3 ? TY + 2 : 1;
  static constexpr int PL = PX * PY;
};

// modes: SW_SMOOTH   out = u + coef (f - A u)
//        SW_SMOOTH2  two sweeps from zero in one: u1 = coef f,
//                    out = u1 + coef (f - A u1) = coef f + coef (f - coef A f)
//        SW_RESID    out = f - A u
//        SW_OUTER    r = F - A v (FP64), out = (TO) r, sums of r^2, F^2
//        SW_SMOOTH_UPD  the last smoothing step of a cycle and the update of
//                    the outer iterate in one: v += (double)(u + coef (f - A u))
//                    (3D tile sweep only)
//        SW_PSMOOTH  the prolongation of the coarse correction and the first
//                    post-smoothing step in one: u' = u + (TS) P e_c at every
//                    staged interior node, out = u' + coef (f - A u')
//                    (3D tile sweep only; u' itself is not stored)
template <typename TS, typename TO, int D, int MODE>
__global__ void __launch_bounds__(256) k_sweep(Ctl ctl, SweepArgs<TS, TO> a) {
  using TT = Tile<D>;
  constexpr int NL = (TT::PL + 255) / 256;     // plane elements per thread
  __shared__ TS pl[3][TT::PL];
  __shared__ double red[MODE == SW_OUTER ? 8 : 1];
  double acc_r = 0.0, acc_f = 0.0;
  const bool active = !skip(ctl);
  if (active) {
    const int m = a.N - 1, n1 = a.n1;
    const int lx = threadIdx.x % TT::TX, ly = threadIdx.x / TT::TX;
    // tiles in XCD-contiguous order: the halo rows a tile shares with its
    // neighbours are then fetched once into that XCD's L2
    const int nbx = gridDim.x, nby = gridDim.y;
    const int lb = kfbi_xcd_block(blockIdx.x + nbx * (blockIdx.y + nby * blockIdx.z), nbx * nby * gridDim.z);
    const int bx = lb % nbx, by = (lb / nbx) % nby, bz = lb / (nbx * nby);
    const int x0 = bx * TT::TX;
    const int y0 = D == 3 ? by * TT::TY : 0;
    const int z0 = (D == 3 ? bz : by) * a.KZ;
    const int z1 = z0 + a.KZ < m ? z0 + a.KZ : m;
    // plane gz into registers (this thread's NL elements), then into LDS
    auto fetch = [&](int gz, TS* r) {
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        const int i = threadIdx.x + 256 * q;
        const int px = i % TT::PX, py = i / TT::PX;
        const int gx = x0 + px, gy = y0 + py;
        TS v = 0;
        if (i < TT::PL && gx <= a.N && (D == 2 || gy <= a.N))
          v = a.s[D == 3 ? gx + n1 * (gy + n1 * gz) : gx + n1 * gz];
        r[q] = v;
      }
    };
    auto store = [&](const TS* r, TS* buf) {
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        const int i = threadIdx.x + 256 * q;
        if (i < TT::PL) buf[i] = r[q];
      }
    };
    // own output node of plane gz (right-hand side value)
    const int ix = x0 + lx, iy = y0 + ly;
    const bool own = ix < m && (D == 2 || iy < m);
    constexpr bool NEEDF = MODE != SW_SMOOTH2;
    auto fetch_f = [&](int gz) -> TS {
      if (!NEEDF || !own) return (TS)0;
      return a.f[D == 3 ? (ix + 1) + n1 * ((iy + 1) + n1 * gz) : (ix + 1) + n1 * gz];
    };
    // two planes in flight: while plane iz+1 is computed, the stencil input
    // of planes iz+3 and iz+4 and the right-hand side of planes iz+2 and
    // iz+3 are being loaded
    TS rA[NL], rB[NL] = {};
    fetch(z0, rA);
    store(rA, pl[z0 % 3]);
    fetch(z0 + 1, rA);
    store(rA, pl[(z0 + 1) % 3]);
    fetch(z0 + 2, rA);
    TS fA = fetch_f(z0 + 1), fB = (TS)0;
    if (z0 + 1 < z1) {
      fetch(z0 + 3, rB);
      fB = fetch_f(z0 + 2);
    }
    const int cc = D == 3 ? (ly + 1) * TT::PX + (lx + 1) : lx + 1;
    for (int iz = z0; iz < z1; ++iz) {
      store(rA, pl[(iz + 2) % 3]);
      __syncthreads();
      TS rC[NL] = {};
      TS fC = (TS)0;
      if (iz + 2 < z1) {
        fetch(iz + 4, rC);
        fC = fetch_f(iz + 3);
      }
      if (own) {
        const TS* P[3] = {pl[iz % 3], pl[(iz + 1) % 3], pl[(iz + 2) % 3]};
        const TS s = stencil_sum<D, TS>(a.c, a.star != 0, [&](int o0, int o1, int o2) {
          return D == 3 ? P[o2 + 1][cc + o1 * TT::PX + o0] : P[o1 + 1][cc + o0];
        });
        const int gz = iz + 1;
        const int idx = D == 3 ? (ix + 1) + n1 * ((iy + 1) + n1 * gz) : (ix + 1) + n1 * gz;
        const TS ctr = P[1][cc];
        if (MODE == SW_SMOOTH) {
          a.out[idx] = (TO)(ctr + a.coef * (fA - s));
        } else if (MODE == SW_SMOOTH2) {
          const TS u1 = a.coef * ctr;
          a.out[idx] = (TO)(u1 + a.coef * (ctr - a.coef * s));
        } else if (MODE == SW_RESID) {
          a.out[idx] = (TO)(fA - s);
        } else {
          const double Fv = (double)fA;
          const double r = Fv - (double)s;
          a.out[idx] = (TO)r;
          acc_r += r * r;
          acc_f += Fv * Fv;
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        rA[q] = rB[q];
        rB[q] = rC[q];
      }
      fA = fB;
      fB = fC;
    }
  }
  if (MODE == SW_OUTER) {
    block_sum2<256>(acc_r, acc_f, red);
    if (threadIdx.x == 0) {
      const int b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
      a.part[b] = acc_r;
      a.part[MG_PART + b] = acc_f;
    }
  }
}

// 3D sweeps, 2.5D blocking.  A workgroup owns a tile of 32 NX (x) by 8 (y)
// nodes of the transverse plane and a chunk of KZ planes; each thread owns
// NX consecutive x nodes of one row.  Input planes stream through two LDS
// buffers (one barrier per plane, the next plane's loads in flight during
// the current plane's arithmetic).  Each input plane p is read from LDS
// once: the thread's 3 x (NX+2) window gives the three in-plane sums
//   Q_o2(p) = sum over (o0, o1) of c[o0 + 3 o1 + 9 o2] u(x+o0-1, y+o1-1, p),
// and out(z) = (Q_0(z-1) + Q_1(z)) + Q_2(z+1) is complete when plane z+1
// has been read.  Same modes as k_sweep.
constexpr int S3_TY = 8;
template <int NX>
struct Tile3 {
  static constexpr int TX = 32 * NX;
  static constexpr int PX = TX + 2, PY = S3_TY + 2;
  static constexpr int PXS = (PX + 3) / 4 * 4;        // LDS row stride (16-byte aligned rows)
  static constexpr int PL = PX * PY;                  // loaded elements per plane
  static constexpr int NL = (PL + 255) / 256;
};

template <typename TS, typename TO, int MODE, int NX>
__global__ void __launch_bounds__(256) k_sweep3(Ctl ctl, SweepArgs<TS, TO> a) {
  using TT = Tile3<NX>;
  __shared__ TS pl[2][TT::PY * TT::PXS];
  __shared__ double red[MODE == SW_OUTER ? 8 : 1];
  double acc_r = 0.0, acc_f = 0.0;
  if (!skip(ctl)) {
    const int m = a.N - 1, n1 = a.n1;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int nbx = gridDim.x, nby = gridDim.y;
    const int lb = kfbi_xcd_block(blockIdx.x + nbx * (blockIdx.y + nby * blockIdx.z), nbx * nby * gridDim.z);
    const int bx = lb % nbx, by = (lb / nbx) % nby, bz = lb / (nbx * nby);
    const int x0 = bx * TT::TX, y0 = by * S3_TY, z0 = bz * a.KZ;
    const int z1 = z0 + a.KZ < m ? z0 + a.KZ : m;
    // output nodes (x0 + NX tx + j + 1, y0 + ty + 1, z), z0 < z <= z1
    const int oy = y0 + ty + 1;
    const bool rowok = oy <= m;
    auto fetch = [&](int gz, TS* r) {
#pragma unroll
      for (int q = 0; q < TT::NL; ++q) {
        const int i = threadIdx.x + 256 * q;
        const int px = i % TT::PX, py = i / TT::PX;
        const int gx = x0 + px, gy = y0 + py;
        r[q] = (i < TT::PL && gx <= a.N && gy <= a.N) ? a.s[gx + (int64_t)n1 * (gy + (int64_t)n1 * gz)] : (TS)0;
      }
    };
    auto store = [&](const TS* r, TS* buf) {
#pragma unroll
      for (int q = 0; q < TT::NL; ++q) {
        const int i = threadIdx.x + 256 * q;
        if (i < TT::PL) buf[(i / TT::PX) * TT::PXS + i % TT::PX] = r[q];
      }
    };
    constexpr bool NEEDF = MODE != SW_SMOOTH2;
    auto fetch_f = [&](int gz, TS* fv) {
#pragma unroll
      for (int j = 0; j < NX; ++j) {
        const int ox = x0 + NX * tx + j + 1;
        fv[j] = (NEEDF && rowok && ox <= m) ? a.f[ox + (int64_t)n1 * (oy + (int64_t)n1 * gz)] : (TS)0;
      }
    };
    TS cur[TT::NL], nxt[TT::NL];
    TS acc0[NX], acc1[NX], ctr0[NX], ctr1[NX], f0[NX], f1[NX];
#pragma unroll
    for (int j = 0; j < NX; ++j) acc0[j] = acc1[j] = ctr0[j] = ctr1[j] = f0[j] = f1[j] = (TS)0;
    fetch(z0, cur);
    for (int p = z0; p <= z1 + 1; ++p) {
      TS* buf = pl[p & 1];
      store(cur, buf);
      __syncthreads();
      if (p + 1 <= z1 + 1) fetch(p + 1, nxt);
      // right-hand side of the output emitted at the next plane (z = p)
      TS fn[NX];
      if (p >= z0 + 1 && p <= z1) fetch_f(p, fn);
      // in-plane window of this thread: rows ty..ty+2, columns NX tx .. NX tx + NX + 1
      TS w[3][NX + 2];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < NX + 2; ++k) w[r][k] = buf[(ty + r) * TT::PXS + NX * tx + k];
#pragma unroll
      for (int j = 0; j < NX; ++j) {
        TS q0 = 0, q1 = 0, q2 = 0;
#pragma unroll
        for (int o1 = 0; o1 < 3; ++o1)
#pragma unroll
          for (int o0 = 0; o0 < 3; ++o0) {
            const TS u = w[o1][j + o0];
            q0 += a.c[o0 + 3 * o1] * u;
            q1 += a.c[o0 + 3 * o1 + 9] * u;
            q2 += a.c[o0 + 3 * o1 + 18] * u;
          }
        const int ox = x0 + NX * tx + j + 1;
        if (p >= z0 + 2 && rowok && ox <= m) {
          // out(p - 1) = (Q_0(p-2) + Q_1(p-1)) + Q_2(p)
          const TS sv = acc1[j] + q2;
          const int64_t idx = ox + (int64_t)n1 * (oy + (int64_t)n1 * (p - 1));
          if (MODE == SW_SMOOTH) {
            a.out[idx] = (TO)(ctr1[j] + a.coef * (f1[j] - sv));
          } else if (MODE == SW_SMOOTH2) {
            const TS u1 = a.coef * ctr1[j];
            a.out[idx] = (TO)(u1 + a.coef * (ctr1[j] - a.coef * sv));
          } else if (MODE == SW_RESID) {
            a.out[idx] = (TO)(f1[j] - sv);
          } else {
            const double Fv = (double)f1[j];
            const double r = Fv - (double)sv;
            a.out[idx] = (TO)r;
            acc_r += r * r;
            acc_f += Fv * Fv;
          }
        }
        acc1[j] = acc0[j] + q1;
        acc0[j] = q0;
        ctr1[j] = w[1][j + 1];
        f1[j] = fn[j];
      }
#pragma unroll
      for (int q = 0; q < TT::NL; ++q) cur[q] = nxt[q];
    }
  }
  if (MODE == SW_OUTER) {
    block_sum2<256>(acc_r, acc_f, red);
    if (threadIdx.x == 0) {
      const int b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
      a.part[b] = acc_r;
      a.part[MG_PART + b] = acc_f;
    }
  }
}

// 3D sweeps on grids up to 128^3, whole tile at once.  At 128^3 a marching
// work group walks only a few planes, one memory round trip after the
// other; here a work group owns 64 x 4 x TZ output nodes, issues the loads
// of its whole (66 x 6 x (TZ+2)) input block and right-hand side at once,
// stages the block in LDS and computes each thread's column of TZ outputs
// from the in-plane partial sums of the planes it passes (the same sums, in
// the same order, as the marching sweep).  Same modes as k_sweep.
constexpr int ST_TX = 64, ST_TY = 4, ST_PX = ST_TX + 2, ST_PY = ST_TY + 2, ST_PXS = 68;

template <typename TS, typename TO, int MODE, int TZ>
__global__ void __launch_bounds__(256) k_sweep3t(Ctl ctl, SweepArgs<TS, TO> a) {
  constexpr int PZ = TZ + 2;
  constexpr int PL = ST_PX * ST_PY * PZ;            // staged input values
  constexpr int NL = (PL + 255) / 256;
  // SW_PSMOOTH: the coarse block under the staged fine block (fine x0 ..
  // x0+65 needs coarse x0/2 .. x0/2+33, likewise 4 in y and z) shares the
  // memory of the staged block (it is dead before the block is written);
  // its interpolation along y and z to the fine planes and rows of the
  // block (at coarse x resolution) follows the block
  constexpr int CX = 34, CY = 4, CZ = 4, NCB = CX * CY * CZ, NYZ = PZ * ST_PY * CX;
  constexpr int BLK_BYTES = PZ * ST_PY * ST_PXS * (int)sizeof(TS);
  static_assert(BLK_BYTES >= NCB * 8, "coarse block larger than the staged block");
  constexpr int EYZ_BYTES = MODE == SW_PSMOOTH ? NYZ * 8 : 0;
  __shared__ __align__(16) unsigned char smem[BLK_BYTES + EYZ_BYTES];
  TS* const blk = (TS*)smem;
  __shared__ double red[MODE == SW_OUTER ? 8 : 1];
  double acc_r = 0.0, acc_f = 0.0;
  if (!skip(ctl)) {
    if (MODE == SW_SMOOTH_UPD && threadIdx.x == 0 && blockIdx.x + blockIdx.y + blockIdx.z == 0)
      a.mctl[1] += 1;   // one more correction applied
    const int m = a.N - 1, n1 = a.n1;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int nbx = gridDim.x, nby = gridDim.y;
    const int lb = kfbi_xcd_block(blockIdx.x + nbx * (blockIdx.y + nby * blockIdx.z), nbx * nby * gridDim.z);
    const int bx = lb % nbx, by = (lb / nbx) % nby, bz = lb / (nbx * nby);
    const int x0 = bx * ST_TX, y0 = by * ST_TY, z0 = bz * TZ;
    // every load of the block and of the right-hand side in flight together
    TS r[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int i = threadIdx.x + 256 * q;
      const int px = i % ST_PX, py = (i / ST_PX) % ST_PY, pz = i / (ST_PX * ST_PY);
      const int gx = x0 + px, gy = y0 + py, gz = z0 + pz;
      r[q] = (i < PL && gx <= a.N && gy <= a.N && gz <= a.N)
                 ? a.s[gx + (int64_t)n1 * (gy + (int64_t)n1 * gz)]
                 : (TS)0;
    }
    const int X0 = x0 / 2, Y0 = y0 / 2, Z0 = z0 / 2;
    constexpr int NCL = MODE == SW_PSMOOTH ? (NCB + 255) / 256 : 1;
    double rc[NCL];
    if constexpr (MODE == SW_PSMOOTH) {
#pragma unroll
      for (int q = 0; q < NCL; ++q) {
        const int i = threadIdx.x + 256 * q;
        const int px = i % CX, py = (i / CX) % CY, pz = i / (CX * CY);
        const int gx = X0 + px, gy = Y0 + py, gz = Z0 + pz;
        rc[q] = (i < NCB && gx <= a.Nc && gy <= a.Nc && gz <= a.Nc)
                    ? a.ec[gx + (int64_t)a.n1c * (gy + (int64_t)a.n1c * gz)]
                    : 0.0;
      }
    }
    const int ox = x0 + tx + 1, oy = y0 + ty + 1;
    const bool colok = ox <= m && oy <= m;
    constexpr bool NEEDF = MODE != SW_SMOOTH2;
    TS fv[TZ];
#pragma unroll
    for (int k = 0; k < TZ; ++k) {
      const int oz = z0 + k + 1;
      fv[k] = (NEEDF && colok && oz <= m) ? a.f[ox + (int64_t)n1 * (oy + (int64_t)n1 * oz)] : (TS)0;
    }
    double* const eyz = (double*)(smem + BLK_BYTES);
    if constexpr (MODE == SW_PSMOOTH) {
      double* const cb = (double*)smem;
#pragma unroll
      for (int q = 0; q < NCL; ++q) {
        const int i = threadIdx.x + 256 * q;
        if (i < NCB) cb[i] = rc[q];
      }
      __syncthreads();
      // along y and z: eyz[pz][py][X] is the average of the coarse values at
      // the (y, z) corners of the coarse cell face / edge that fine row
      // (y0 + py, z0 + pz) lies on, at coarse x = X0 + X (the reciprocal of
      // the count is exact; all four corners lie in the coarse block and
      // the ones off the face add zero)
      for (int i = threadIdx.x; i < NYZ; i += 256) {
        const int X = i % CX, py = (i / CX) % ST_PY, pz = i / (CX * ST_PY);
        const int gy = y0 + py, gz = z0 + pz;
        const int p1 = gy & 1, p2 = gz & 1;
        const double* cq = cb + X + CX * (((gy >> 1) - Y0) + CY * ((gz >> 1) - Z0));
        const double c00 = cq[0], c01 = cq[CX], c10 = cq[CX * CY], c11 = cq[CX * CY + CX];
        double sc = c00;
        sc += p1 ? c01 : 0.0;
        sc += p2 ? c10 : 0.0;
        sc += (p1 && p2) ? c11 : 0.0;
        eyz[i] = sc * (1.0 / (double)(1 << (p1 + p2)));
      }
      __syncthreads();   // the staged block overwrites cb below
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int i = threadIdx.x + 256 * q;
      if (i < PL) {
        const int px = i % ST_PX, py = (i / ST_PX) % ST_PY, pz = i / (ST_PX * ST_PY);
        blk[(pz * ST_PY + py) * ST_PXS + px] = r[q];
      }
    }
    __syncthreads();
    if constexpr (MODE == SW_PSMOOTH) {
      // then along x: u' = u + (TS) P e_c at the interior nodes of the block
      // (the box boundary keeps its zero), in place in the staged block
      for (int i = threadIdx.x; i < PL; i += 256) {
        const int px = i % ST_PX, py = (i / ST_PX) % ST_PY, pz = i / (ST_PX * ST_PY);
        const int gx = x0 + px, gy = y0 + py, gz = z0 + pz;
        if (gx >= 1 && gx <= m && gy >= 1 && gy <= m && gz >= 1 && gz <= m) {
          const double* eq = eyz + ((gx >> 1) - X0) + CX * (py + ST_PY * pz);
          const double sc = (gx & 1) ? (eq[0] + eq[1]) * 0.5 : eq[0];
          TS* const bq = blk + (pz * ST_PY + py) * ST_PXS + px;
          *bq = *bq + (TS)sc;
        }
      }
      __syncthreads();
    }
    TS acc0 = 0, acc1 = 0, ctr = 0;   // ctr: centre value of the previous plane
#pragma unroll
    for (int p = 0; p < PZ; ++p) {
      const TS* pl = blk + p * ST_PY * ST_PXS;
      TS q0 = 0, q1 = 0, q2 = 0;
#pragma unroll
      for (int o1 = 0; o1 < 3; ++o1)
#pragma unroll
        for (int o0 = 0; o0 < 3; ++o0) {
          const TS u = pl[(ty + o1) * ST_PXS + tx + o0];
          q0 += a.c[o0 + 3 * o1] * u;
          q1 += a.c[o0 + 3 * o1 + 9] * u;
          q2 += a.c[o0 + 3 * o1 + 18] * u;
        }
      if (p >= 2) {
        // output k = p - 2 at plane z0 + p - 1: (Q_0(p-2) + Q_1(p-1)) + Q_2(p)
        const int k = p - 2;
        const int oz = z0 + k + 1;
        if (colok && oz <= m) {
          const TS sv = acc1 + q2;
          const int64_t idx = ox + (int64_t)n1 * (oy + (int64_t)n1 * oz);
          if (MODE == SW_SMOOTH || MODE == SW_PSMOOTH) {
            a.out[idx] = (TO)(ctr + a.coef * (fv[k] - sv));
          } else if (MODE == SW_SMOOTH2) {
            const TS u1 = a.coef * ctr;
            a.out[idx] = (TO)(u1 + a.coef * (ctr - a.coef * sv));
          } else if (MODE == SW_RESID) {
            a.out[idx] = (TO)(fv[k] - sv);
          } else if (MODE == SW_SMOOTH_UPD) {
            a.v[idx] = a.v[idx] + (double)(ctr + a.coef * (fv[k] - sv));
          } else {
            const double Fv = (double)fv[k];
            const double rr = Fv - (double)sv;
            a.out[idx] = (TO)rr;
            acc_r += rr * rr;
            acc_f += Fv * Fv;
          }
        }
      }
      acc1 = acc0 + q1;
      acc0 = q0;
      ctr = pl[(ty + 1) * ST_PXS + tx + 1];
    }
  }
  if (MODE == SW_OUTER) {
    block_sum2<256>(acc_r, acc_f, red);
    if (threadIdx.x == 0) {
      const int b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
      a.part[b] = acc_r;
      a.part[MG_PART + b] = acc_f;
    }
  }
}

// coarse right-hand side f_c = R r_f, formed in T and stored in FP64
template <typename T>
__global__ void __launch_bounds__(MG_BLOCK) k_restrict(Ctl ctl, Lev<T> Fl, int Nc, int n1c, const T* r, double* fc) {
  if (skip(ctl)) return;
  const int64_t m = Fl.d == 3 ? (int64_t)(Nc - 1) * (Nc - 1) * (Nc - 1) : (int64_t)(Nc - 1) * (Nc - 1);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
    int I0, I1, I2;
    node_ijk(Fl.d, t, Nc, I0, I1, I2);
    const int64_t idx = I0 + (int64_t)n1c * (I1 + (int64_t)n1c * I2);
    fc[idx] = (double)op_restrict<T>(Fl.d, Fl.n1, r, I0, I1, I2);
  }
}

// u_f += (T) P e_c at the fine interior (interpolation in FP64)
template <typename T>
__global__ void __launch_bounds__(MG_BLOCK) k_prolong(Ctl ctl, Lev<T> Fl, int n1c, const double* ec, T* u) {
  if (skip(ctl)) return;
  const int64_t m = Fl.d == 3 ? (int64_t)(Fl.N - 1) * (Fl.N - 1) * (Fl.N - 1) : (int64_t)(Fl.N - 1) * (Fl.N - 1);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
    int i0, i1, i2;
    node_ijk(Fl.d, t, Fl.N, i0, i1, i2);
    const int64_t idx = i0 + (int64_t)Fl.n1 * (i1 + (int64_t)Fl.n1 * i2);
    u[idx] += (T)op_prolong<double>(Fl.d, n1c, ec, i0, i1, i2);
  }
}

// ---------------------------------------------------------------- box-solution store
// slot 1 + j of GMRES iteration j (control word; nothing once GMRES has
// converged or beyond the slots) or slot 0 (no control word)
__global__ void __launch_bounds__(MG_BLOCK) k_ustore(const int* gctl, int64_t n, int slots, const double* v,
                                                    double* store) {
  int slot = 0;
  if (gctl) {
    if (gctl[1]) return;
    slot = 1 + gctl[0];
    if (slot >= slots) return;
  }
  double* dst = store + (int64_t)slot * n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    dst[t] = v[t];
}

// v = (use_x0 ? slot 0 : 0) + sum_{j < k} y_j slot(1 + j)
__global__ void __launch_bounds__(MG_BLOCK) k_ucombine(int64_t n, int k, int use_x0, const double* y,
                                                      const double* store, double* v) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    double s = use_x0 ? store[t] : 0.0;
    for (int j = 0; j < k; ++j) s += y[j] * store[(int64_t)(1 + j) * n + t];
    v[t] = s;
  }
}

__global__ void __launch_bounds__(MG_BLOCK) k_usum(int64_t n, const double* a, const double* b, double* out) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    out[t] = a[t] + b[t];
}

__global__ void __launch_bounds__(MG_BLOCK) k_udiff(int64_t n, const double* a, const double* b, double* out) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    out[t] = a[t] - b[t];
}

__global__ void __launch_bounds__(MG_BLOCK) k_uzero(int64_t n, double* v) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    v[t] = 0.0;
}

// ---------------------------------------------------------------- FP64 outer loop
struct OuterArgs {
  Ctl ctl;
  int d, N, n1;
  double c[27];
  const double* F;
  double* v;
  int first;          // v = 0 (written here): r = F, and |F| is accumulated too
  double* part;       // [2][MG_PART]
};

// first correction (v = 0): v <- 0, f_0 = (T) F; per-block sums of F^2
// (later corrections use the SW_OUTER sweep)
template <typename T>
__global__ void __launch_bounds__(MG_BLOCK) k_outer_resid(OuterArgs a, T* f0) {
  __shared__ double red[2 * MG_BLOCK / 64];
  double acc_r = 0.0, acc_f = 0.0;
  if (!skip(a.ctl)) {
    const int64_t m = a.d == 3 ? (int64_t)(a.N - 1) * (a.N - 1) * (a.N - 1) : (int64_t)(a.N - 1) * (a.N - 1);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
      const int64_t idx = node_of(a.d, a.n1, t, a.N);
      const double Fv = a.F[idx];
      const double r = Fv;     // first correction: v = 0
      a.v[idx] = 0.0;
      f0[idx] = (T)r;
      acc_r += r * r;
      acc_f += Fv * Fv;
    }
  }
  block_sum2<MG_BLOCK>(acc_r, acc_f, red);
  if (threadIdx.x == 0) {
    a.part[blockIdx.x] = acc_r;
    a.part[MG_PART + blockIdx.x] = acc_f;
  }
}

// stopping test: |r| <= eps |F| (|F| taken at the first correction).
// Relaxed inner tolerance inside a captured GMRES iteration: the box solve
// of the matvec at GMRES step j only needs an accuracy in proportion to
// tol |b| / |r_j| (inexact Krylov), so eps becomes relax tol |b| / |r_j|
// from the GMRES scalars (gs[0] = |r_j| estimate, gs[1] = |b|, gs[3] =
// tol, gs[7] = relax, 0 for off), clamped to [eps, 1e-1] (one correction
// of the two-grid cycle, which contracts by 0.07, reaches 1e-1).
__global__ void __launch_bounds__(CHECK_BLOCK) k_check(Ctl ctl, const double* part, int nblk, int first,
                                                      double eps, int maxit, double* scal, const double* gs,
                                                      int count_hit) {
  if ((ctl.gctl && ctl.gctl[1]) || ctl.mctl[0]) return;
  const double relax = (ctl.gctl && gs) ? gs[7] : 0.0;
  if (relax > 0.0) {
    const double rj = gs[0], nb = gs[1], tol = gs[3];
    if (rj > 0.0 && nb > 0.0) {
      double e = relax * tol * nb / rj;
      if (e > 1e-1) e = 1e-1;
      if (e > eps) eps = e;
    }
  }
  __shared__ double red[2 * CHECK_BLOCK / 64];
  double r = 0.0, f = 0.0;
  for (int i = threadIdx.x; i < nblk; i += CHECK_BLOCK) {
    r += part[i];
    f += part[MG_PART + i];
  }
  block_sum2<CHECK_BLOCK>(r, f, red);
  if (threadIdx.x == 0) {
    if (first) scal[0] = sqrt(f);
    const double nr = sqrt(r);
    const double nf = scal[0];
    const double rel = nf > 0.0 ? nr / nf : 0.0;
    scal[1] = rel;
    const bool conv = rel <= eps || nf == 0.0;
    if (conv || ctl.mctl[1] >= maxit) {
      ctl.mctl[0] = 1;
      if (ctl.mctl[1] > ctl.mctl[2]) ctl.mctl[2] = ctl.mctl[1];
      // a box solve stopped by its cap above eps_in (the relaxed iterations
      // keep a record of their own, mctl[4 + j])
      if (!conv && !(relax > 0.0) && count_hit) ctl.mctl[3] += 1;
      if (ctl.gctl) ctl.mctl[4 + ctl.gctl[0]] = ctl.mctl[1];   // corrections of GMRES iteration j
    }
  }
}

// v += e, interior only
template <typename T>
__global__ void __launch_bounds__(MG_BLOCK) k_update(Ctl ctl, int d, int N, int n1, const T* e, double* v) {
  if (skip(ctl)) return;
  // every node, boundary included: the correction is zero on the box
  // boundary (the level arrays never write it), so a plain stream
  const int64_t m = d == 3 ? (int64_t)n1 * n1 * n1 : (int64_t)n1 * n1;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl.mctl[1] += 1;   // one more correction applied
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x)
    v[t] = v[t] + (double)e[t];
}

// v = 0 on the box boundary (the outer residual reads v's boundary nodes;
// the caller's buffer may hold box data there)
__global__ void __launch_bounds__(MG_BLOCK) k_zero_boundary(Ctl ctl, int d, int n1, double* v) {
  if (ctl.gctl && ctl.gctl[1]) return;
  const int64_t face = d == 3 ? (int64_t)n1 * n1 : (int64_t)n1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * d * face) return;
  const int f = (int)(t / face);          // axis f / 2, side f % 2
  const int64_t r = t % face;
  const int ax = f >> 1;
  const int side = (f & 1) ? n1 - 1 : 0;
  int c[3] = {0, 0, 0};
  int o[2] = {(int)(r % n1), (int)(r / n1)};
  int q = 0;
  for (int a = 0; a < d; ++a) c[a] = a == ax ? side : o[q++];
  v[c[0] + (int64_t)n1 * (c[1] + (int64_t)n1 * c[2])] = 0.0;
}

__global__ void k_start(Ctl ctl) {
  if (ctl.gctl && ctl.gctl[1]) return;
  ctl.mctl[0] = 0;
  ctl.mctl[1] = 0;
}

// right-hand side of the matvec: F = -sum over cut neighbours Q of
// A_PQ (C^(reg P) - C^(reg Q))(x_Q) at the irregular nodes (the nodes are
// fixed per plan; F is zero elsewhere)
__global__ void __launch_bounds__(MG_BLOCK) k_scatter(const int* gctl, int64_t n_irr, int maxpairs, const int* irr,
                                                     const double* PA, const int* PE1, const int* PE2,
                                                     const double* Cv, double* F) {
  if (gctl && gctl[1]) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_irr) return;
  double s = 0.0;
  for (int m = 0; m < maxpairs; ++m) {
    const double cf = PA[t * maxpairs + m];
    if (cf == 0.0) break;
    const int e1 = PE1[t * maxpairs + m], e2 = PE2[t * maxpairs + m];
    const double c1 = e1 >= 0 ? Cv[e1] : 0.0, c2 = e2 >= 0 ? Cv[e2] : 0.0;
    s -= cf * (c1 - c2);
  }
  F[irr[t]] = s;
}

inline unsigned nblk(int64_t n, int b = MG_BLOCK) { return (unsigned)((n + b - 1) / b); }
// grid of an elementwise grid-stride kernel: enough workgroups to fill the
// chip, few enough that a launch skipped by the control word is cheap
inline unsigned gsblk(int64_t n) {
  unsigned b = nblk(n);
  return b > 4096u ? 4096u : b;
}

// the fine grid's operator, smoother and layout
template <typename T>
Lev<T> fine_level(const kfbi_plan* pl) {
  Lev<T> L;
  L.N = pl->g.N;
  L.n1 = L.N + 1;
  L.d = pl->g.d;
  L.off = 0;
  for (int i = 0; i < 27; ++i) L.c[i] = (T)pl->mg_c[i];
  L.coef = (T)(pl->mg_w / pl->mg_c[13]);   // central coefficient: offset (0,0,0)
  L.inva = (T)(1.0 / pl->mg_c[13]);
  L.star = stencil_is_star(pl->mg_c);
  return L;
}

struct SweepGeom {
  dim3 grid;
  int KZ;
  int blocks;
};

// tiles of the transverse plane x chunks of KZ planes, about 1024 workgroups
template <int D>
SweepGeom sweep_geom(int N) {
  using TT = Tile<D>;
  const int m = N - 1;
  const int tx = (m + TT::TX - 1) / TT::TX;
  const int ty = D == 3 ? (m + TT::TY - 1) / TT::TY : 1;
  const int cols = tx * ty;
  int chunks = 4096 / cols;
  if (chunks < 1) chunks = 1;
  int KZ = (m + chunks - 1) / chunks;
  const int kmin = D == 3 ? 8 : 8;
  if (KZ < kmin) KZ = kmin;
  if (KZ > m) KZ = m;
  chunks = (m + KZ - 1) / KZ;
  SweepGeom g;
  g.grid = D == 3 ? dim3(tx, ty, chunks) : dim3(tx, chunks, 1);
  g.KZ = KZ;
  g.blocks = cols * chunks;
  return g;
}

// 3D: tiles of 64 x 8 nodes (2 x nodes per thread) x chunks of KZ >= 4
// planes, about 2048 workgroups (measured at 128^3 and 256^3, FP32 and
// FP64), never more than the MG_PART partial-sum slots
constexpr int S3_NX = 2;
inline SweepGeom sweep3_geom(int N) {
  const int m = N - 1;
  const int tx = (m + 32 * S3_NX - 1) / (32 * S3_NX), ty = (m + S3_TY - 1) / S3_TY;
  const int tiles = tx * ty;
  int chunks = 2048 / tiles;
  if (chunks < 1) chunks = 1;
  int KZ = (m + chunks - 1) / chunks;
  if (KZ < 4) KZ = 4;
  if (KZ > m) KZ = m;
  while ((int64_t)tiles * ((m + KZ - 1) / KZ) > MG_PART) KZ *= 2;
  if (KZ > m) KZ = m;
  SweepGeom g;
  g.KZ = KZ;
  g.grid = dim3(tx, ty, (m + KZ - 1) / KZ);
  g.blocks = tiles * ((m + KZ - 1) / KZ);
  return g;
}

template <typename TS, typename TO, int MODE>
void sweep(kfbi_plan* pl, Ctl ctl, int N, const TS* c27, TS coef, const TS* src, const TS* f, TO* out,
           int* nblocks = nullptr, double* v = nullptr) {
  SweepArgs<TS, TO> a;
  a.v = v;
  a.mctl = ctl.mctl;
  a.N = N;
  a.n1 = N + 1;
  double cd[27];
  for (int i = 0; i < 27; ++i) {
    a.c[i] = c27[i];
    cd[i] = (double)c27[i];
  }
  a.star = stencil_is_star(cd);
  a.coef = coef;
  a.s = src;
  a.f = f;
  a.out = out;
  a.part = pl->mg_part;
  a.ec = pl->mg_Uc;
  a.Nc = pl->mg_gc.N;
  a.n1c = pl->mg_gc.n1;
  if constexpr (MODE == SW_SMOOTH_UPD || MODE == SW_PSMOOTH) {
    // the tile sweep only (the caller's grid is 3D with N <= 128)
    const int m = N - 1;
    const dim3 grid((m + ST_TX - 1) / ST_TX, (m + ST_TY - 1) / ST_TY, (m + 3) / 4);
    a.KZ = 4;
    hipLaunchKernelGGL((k_sweep3t<TS, TO, MODE, 4>), grid, dim3(256), 0, pl->stream, ctl, a);
    if (nblocks) *nblocks = (int)(grid.x * grid.y * grid.z);
  } else if (pl->g.d == 3 && N <= 128) {
    // whole tile at once: 64 x 4 x 4 outputs per work group (2048 at 128^3)
    const int m = N - 1;
    const dim3 grid((m + ST_TX - 1) / ST_TX, (m + ST_TY - 1) / ST_TY, (m + 3) / 4);
    a.KZ = 4;
    hipLaunchKernelGGL((k_sweep3t<TS, TO, MODE, 4>), grid, dim3(256), 0, pl->stream, ctl, a);
    if (nblocks) *nblocks = (int)(grid.x * grid.y * grid.z);
  } else if (pl->g.d == 3) {
    SweepGeom g = sweep3_geom(N);
    a.KZ = g.KZ;
    hipLaunchKernelGGL((k_sweep3<TS, TO, MODE, S3_NX>), g.grid, dim3(256), 0, pl->stream, ctl, a);
    if (nblocks) *nblocks = g.blocks;
  } else {
    SweepGeom g = sweep_geom<2>(N);
    a.KZ = g.KZ;
    hipLaunchKernelGGL((k_sweep<TS, TO, 2, MODE>), g.grid, dim3(256), 0, pl->stream, ctl, a);
    if (nblocks) *nblocks = g.blocks;
  }
}

// the fused kernels cover 3D grids up to 128^3 (partial sums and tile counts)
inline bool fused_path(const kfbi_plan* pl) { return pl->g.d == 3 && pl->g.N <= 128; }

// the exact FP64 solve of the coarse grid (tracing aid, profile mode 3:
// events around its passes in eager box solves)
void coarse_solve(kfbi_plan* pl, Ctl ctl, hipStream_t st, const void* rsrc = nullptr, int rsrc_f32 = 0) {
  const GridDesc& gc = pl->mg_gc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (pl->prof_on == 3 && pl->prof_ev && !pl->ctl_active) {
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess)
      (void)hipEventRecord(e0, st);
    else
      e0 = e1 = nullptr;
  }
  dst_solve_grid(gc, pl->mg_twc, pl->mg_eigc, pl->mg_T1c, pl->mg_T2c, pl->mg_Fc, pl->mg_Uc, ctl.gctl, ctl.mctl, st,
                 rsrc, rsrc_f32, pl->g.n1);
  if (e0 && e1) {
    (void)hipEventRecord(e1, st);
    pl->prof_ev->push_back(e0);
    pl->prof_ev->push_back(e1);
    pl->prof_launches += gc.d == 3 ? 5 : 3;
  }
}

// one two-grid cycle with the update v += e folded into the last smoothing
// sweep (3D, N <= 128: the whole-tile sweeps)
template <typename T>
void vcycle_fused(kfbi_plan* pl, const Lev<T>& L, Ctl ctl, double* v) {
  T* u = (T*)pl->mg_u;
  T* tb = (T*)pl->mg_t;
  T* f = (T*)pl->mg_f;
  hipStream_t st = pl->stream;
  sweep<T, T, SW_SMOOTH2>(pl, ctl, L.N, L.c, L.coef, f, f, u);
  sweep<T, T, SW_RESID>(pl, ctl, L.N, L.c, L.coef, u, f, tb);
  // the restriction of the residual is formed by the coarse solve's first
  // pass as it loads its lines
  coarse_solve(pl, ctl, st, (const void*)tb, sizeof(T) == 4 ? 1 : 0);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (pl->prof_on == 2 && pl->prof_ev && !pl->ctl_active) {
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess)
      (void)hipEventRecord(e0, st);
    else
      e0 = e1 = nullptr;
  }
  // the prolongation of the coarse correction inside the first
  // post-smoothing step (the prolonged u is not stored)
  sweep<T, T, SW_PSMOOTH>(pl, ctl, L.N, L.c, L.coef, u, f, tb);
  if (e0 && e1) {
    (void)hipEventRecord(e1, st);
    pl->prof_ev->push_back(e0);
    pl->prof_ev->push_back(e1);
    pl->prof_launches += 1;
  }
  sweep<T, T, SW_SMOOTH_UPD>(pl, ctl, L.N, L.c, L.coef, tb, f, u, nullptr, v);
}

template <typename T>
void vcycle(kfbi_plan* pl, const Lev<T>& L, Ctl ctl) {
  T* u = (T*)pl->mg_u;
  T* tb = (T*)pl->mg_t;
  T* f = (T*)pl->mg_f;
  hipStream_t st = pl->stream;
  const GridDesc& gc = pl->mg_gc;
  const int64_t mf = L.d == 3 ? (int64_t)(L.N - 1) * (L.N - 1) * (L.N - 1) : (int64_t)(L.N - 1) * (L.N - 1);
  const int64_t mc = L.d == 3 ? (int64_t)(gc.N - 1) * (gc.N - 1) * (gc.N - 1) : (int64_t)(gc.N - 1) * (gc.N - 1);
  sweep<T, T, SW_SMOOTH2>(pl, ctl, L.N, L.c, L.coef, f, f, u);
  sweep<T, T, SW_RESID>(pl, ctl, L.N, L.c, L.coef, u, f, tb);
  hipLaunchKernelGGL((k_restrict<T>), dim3(gsblk(mc)), dim3(MG_BLOCK), 0, st, ctl, L, gc.N, gc.n1, (const T*)tb,
                     pl->mg_Fc);
  coarse_solve(pl, ctl, st);
  hipLaunchKernelGGL((k_prolong<T>), dim3(gsblk(mf)), dim3(MG_BLOCK), 0, st, ctl, L, gc.n1,
                     (const double*)pl->mg_Uc, u);
  // tracing aid (profile mode 2, eager solves only): events around the
  // two post-smoothing sweeps
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (pl->prof_on == 2 && pl->prof_ev && !pl->ctl_active) {
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess)
      (void)hipEventRecord(e0, st);
    else
      e0 = e1 = nullptr;
  }
  sweep<T, T, SW_SMOOTH>(pl, ctl, L.N, L.c, L.coef, u, f, tb);
  sweep<T, T, SW_SMOOTH>(pl, ctl, L.N, L.c, L.coef, tb, f, u);
  if (e0 && e1) {
    (void)hipEventRecord(e1, st);
    pl->prof_ev->push_back(e0);
    pl->prof_ev->push_back(e1);
    pl->prof_launches += 2;
  }
}

template <typename T>
void solve_t(kfbi_plan* pl, const double* F, double* v) {
  const Lev<T> L = fine_level<T>(pl);
  Ctl ctl{pl->ctl_active, pl->mg_ctl};
  hipStream_t st = pl->stream;
  const GridDesc& g = pl->g;
  const int64_t m = g.d == 3 ? (int64_t)(g.N - 1) * (g.N - 1) * (g.N - 1) : (int64_t)(g.N - 1) * (g.N - 1);
  unsigned gout = nblk(m);
  if (gout > (unsigned)MG_PART) gout = MG_PART;
  OuterArgs oa;
  oa.ctl = ctl;
  oa.d = g.d;
  oa.N = g.N;
  oa.n1 = g.n1;
  for (int i = 0; i < 27; ++i) oa.c[i] = pl->mg_c[i];
  oa.F = F;
  oa.v = v;
  oa.part = pl->mg_part;
  oa.first = 1;
  // from a given v (its box boundary zero like every stored solution) the
  // first correction takes the full outer residual too, and a stop at the
  // cap is no sign of a short cap (the caller continues such a solve)
  const bool guess = pl->mg_guess;
  hipLaunchKernelGGL(k_start, dim3(1), dim3(1), 0, st, ctl);
  {
    const int64_t nb = 2 * g.d * (g.d == 3 ? (int64_t)g.n1 * g.n1 : (int64_t)g.n1);
    hipLaunchKernelGGL(k_zero_boundary, dim3(nblk(nb)), dim3(MG_BLOCK), 0, st, ctl, g.d, g.n1, v);
  }
  T* f0 = (T*)pl->mg_f;
  const int cap = pl->mg_run_cap > 0 ? pl->mg_run_cap : pl->mg_maxit;
  for (int it = 0; it < cap; ++it) {
    int nb_part = (int)gout;
    if (it == 0 && !guess)
      hipLaunchKernelGGL((k_outer_resid<T>), dim3(gout), dim3(MG_BLOCK), 0, st, oa, f0);
    else
      sweep<double, T, SW_OUTER>(pl, ctl, g.N, pl->mg_c, 0.0, v, F, f0, &nb_part);
    hipLaunchKernelGGL(k_check, dim3(1), dim3(CHECK_BLOCK), 0, st, ctl, (const double*)pl->mg_part, nb_part,
                       it == 0 ? 1 : 0, pl->mg_eps, cap, pl->mg_scal, (const double*)pl->scal, guess ? 0 : 1);
    if (fused_path(pl)) {
      vcycle_fused<T>(pl, L, ctl, v);
    } else {
      vcycle<T>(pl, L, ctl);
      hipLaunchKernelGGL((k_update<T>), dim3(gsblk(m)), dim3(MG_BLOCK), 0, st, ctl, g.d, g.N, g.n1,
                         (const T*)pl->mg_u, v);
    }
  }
  // residual of the final iterate (the stopping value reported)
  int nb_part = 0;
  sweep<double, T, SW_OUTER>(pl, ctl, g.N, pl->mg_c, 0.0, v, F, f0, &nb_part);
  hipLaunchKernelGGL(k_check, dim3(1), dim3(CHECK_BLOCK), 0, st, ctl, (const double*)pl->mg_part, nb_part, 0,
                     pl->mg_eps, cap, pl->mg_scal, (const double*)pl->scal, guess ? 0 : 1);
}

double jacobi_weight(const double* c, int d) {
  // range of lambda(theta)/a over the high frequencies on a 64^d sample grid
  const int S = 64;
  const double a = c[13];
  double lo = 1e300, hi = -1e300;
  const int nz = d == 3 ? S : 1;
  for (int k2 = 1; k2 <= nz; ++k2)
    for (int k1 = 1; k1 <= S; ++k1)
      for (int k0 = 1; k0 <= S; ++k0) {
        const double t0 = M_PI * k0 / S, t1 = M_PI * k1 / S, t2 = d == 3 ? M_PI * k2 / S : 0.0;
        double tm = t0 > t1 ? t0 : t1;
        if (d == 3 && t2 > tm) tm = t2;
        if (tm < M_PI / 2) continue;
        double lam = 0.0;
        const int zr = d == 3 ? 1 : 0;
        for (int o2 = -zr; o2 <= zr; ++o2)
          for (int o1 = -1; o1 <= 1; ++o1)
            for (int o0 = -1; o0 <= 1; ++o0) {
              const double cf = c[(o0 + 1) + 3 * (o1 + 1) + 9 * (o2 + 1)];
              if (cf != 0.0) lam += cf * cos(o0 * t0 + o1 * t1 + o2 * t2);
            }
        const double rho = lam / a;
        lo = rho < lo ? rho : lo;
        hi = rho > hi ? rho : hi;
      }
  return 2.0 / (lo + hi);
}

}  // namespace

// stencil of A_h (operator.hip)
void kfbi_stencil_A(const GridDesc& g, double* A27);

kfbi_status mg_configure(kfbi_plan* pl, int solver, double eps, int maxit) {
  pl->box_solver = solver;
  pl->mg_eps = eps;
  pl->mg_maxit = maxit;
  pl->mg_cap_eff = 0;
  pl->mg_run_cap = 0;
  pl->mg_guess = false;
  if (solver == KFBI_BOX_FFT) return KFBI_OK;
  const GridDesc& g = pl->g;
  if (g.N < 16) {
    kfbi_set_error("the multigrid box solver needs N >= 16 (coarse grid N/2 >= 8; got N = %d)", g.N);
    return KFBI_E_INVALID;
  }
  kfbi_stencil_A(g, pl->mg_c);
  pl->mg_w = jacobi_weight(pl->mg_c, g.d);
  // coarse grid of the two-grid cycle: same operator with 2h
  GridDesc gc = g;
  gc.N = g.N / 2;
  gc.n1 = gc.N + 1;
  gc.h = 2.0 * g.h;
  gc.n_nodes = 1;
  for (int a = 0; a < g.d; ++a) gc.n_nodes *= gc.n1;
  pl->mg_gc = gc;
  const size_t es = solver == KFBI_BOX_MG32 ? sizeof(float) : sizeof(double);
  const int64_t nf = g.n_nodes;
  if (nf * (int64_t)es > pl->mg_bytes) {
    if (pl->mg_u) (void)hipFree(pl->mg_u);
    if (pl->mg_t) (void)hipFree(pl->mg_t);
    if (pl->mg_f) (void)hipFree(pl->mg_f);
    pl->mg_u = pl->mg_t = pl->mg_f = nullptr;
    pl->mg_bytes = 0;
    const size_t b = (size_t)nf * es;
    if (hipMalloc(&pl->mg_u, b) != hipSuccess || hipMalloc(&pl->mg_t, b) != hipSuccess ||
        hipMalloc(&pl->mg_f, b) != hipSuccess) {
      (void)hipGetLastError();
      kfbi_set_error("device allocation of the multigrid grids failed");
      return KFBI_E_OOM;
    }
    pl->mg_bytes = (int64_t)b;
  }
  // zero boundaries once; the kernels only write interiors
  HIPCHK(hipMemsetAsync(pl->mg_u, 0, (size_t)pl->mg_bytes, pl->stream));
  HIPCHK(hipMemsetAsync(pl->mg_t, 0, (size_t)pl->mg_bytes, pl->stream));
  HIPCHK(hipMemsetAsync(pl->mg_f, 0, (size_t)pl->mg_bytes, pl->stream));
  if (gc.n_nodes > pl->mg_nc) {
    double** bufs[4] = {&pl->mg_Fc, &pl->mg_Uc, &pl->mg_T1c, &pl->mg_T2c};
    for (double** b : bufs) {
      if (*b) (void)hipFree(*b);
      *b = nullptr;
    }
    if (pl->mg_twc) (void)hipFree(pl->mg_twc);
    if (pl->mg_eigc) (void)hipFree(pl->mg_eigc);
    pl->mg_twc = pl->mg_eigc = nullptr;
    pl->mg_nc = 0;
    for (double** b : bufs)
      if (hipMalloc((void**)b, sizeof(double) * gc.n_nodes) != hipSuccess) {
        (void)hipGetLastError();
        kfbi_set_error("device allocation of the multigrid coarse grid failed");
        return KFBI_E_OOM;
      }
    if (hipMalloc((void**)&pl->mg_twc, sizeof(double) * 4 * gc.N) != hipSuccess ||
        hipMalloc((void**)&pl->mg_eigc, sizeof(double) * (gc.N + 1)) != hipSuccess) {
      (void)hipGetLastError();
      kfbi_set_error("device allocation of the coarse transform tables failed");
      return KFBI_E_OOM;
    }
    pl->mg_nc = gc.n_nodes;
  }
  // the coarse solution's box boundary stays zero (the passes write interiors)
  HIPCHK(hipMemsetAsync(pl->mg_Uc, 0, sizeof(double) * gc.n_nodes, pl->stream));
  HIPCHK(hipMemsetAsync(pl->mg_Fc, 0, sizeof(double) * gc.n_nodes, pl->stream));
  {
    std::vector<double> tw((size_t)4 * gc.N), eig((size_t)gc.N + 1);
    dst_host_tables(gc.N, gc.h, tw.data(), eig.data());
    HIPCHK(hipMemcpyAsync(pl->mg_twc, tw.data(), sizeof(double) * tw.size(), hipMemcpyHostToDevice, pl->stream));
    HIPCHK(hipMemcpyAsync(pl->mg_eigc, eig.data(), sizeof(double) * eig.size(), hipMemcpyHostToDevice, pl->stream));
    HIPCHK(hipStreamSynchronize(pl->stream));   // the host tables go out of scope
  }
  KCHK(dst_autotune_grid(gc, pl->mg_twc, pl->mg_eigc, pl->mg_T1c, pl->mg_T2c, pl->stream));
  if (!pl->mg_part) {
    if (hipMalloc((void**)&pl->mg_part, sizeof(double) * 2 * MG_PART) != hipSuccess ||
        hipMalloc((void**)&pl->mg_ctl, sizeof(int) * (4 + KFBI_GMRES_MAX + 2)) != hipSuccess ||
        hipMalloc((void**)&pl->mg_scal, sizeof(double) * 4) != hipSuccess) {
      (void)hipGetLastError();
      kfbi_set_error("device allocation of the multigrid control failed");
      return KFBI_E_OOM;
    }
    HIPCHK(hipMemsetAsync(pl->mg_ctl, 0, sizeof(int) * (4 + KFBI_GMRES_MAX + 2), pl->stream));
    HIPCHK(hipMemsetAsync(pl->mg_scal, 0, sizeof(double) * 4, pl->stream));
  }
  if (!pl->Fmg) {
    if (hipMalloc((void**)&pl->Fmg, sizeof(double) * g.n_nodes) != hipSuccess) {
      (void)hipGetLastError();
      kfbi_set_error("device allocation of the multigrid right-hand side failed");
      return KFBI_E_OOM;
    }
  }
  HIPCHK(hipMemsetAsync(pl->Fmg, 0, sizeof(double) * g.n_nodes, pl->stream));
  HIPCHK(hipStreamSynchronize(pl->stream));
  return KFBI_OK;
}

namespace {
void solve_enqueue(kfbi_plan* pl, const double* F, double* v) {
  if (pl->box_solver == KFBI_BOX_MG32)
    solve_t<float>(pl, F, v);
  else
    solve_t<double>(pl, F, v);
}

// everything the kernels of a captured solve take by value or by address,
// other than F, v, the control word, the cap and the start
void config_key(const kfbi_plan* pl, uint64_t* key) {
  memset(key, 0, sizeof(uint64_t) * 48);
  int i = 0;
  auto put = [&](uint64_t x) { key[i++] = x; };
  auto putd = [&](double x) {
    uint64_t u;
    memcpy(&u, &x, 8);
    put(u);
  };
  put((uint64_t)pl->g.d | (uint64_t)pl->g.N << 8 | (uint64_t)pl->box_solver << 40);
  putd(pl->mg_w);
  for (int c = 0; c < 27; ++c) putd(pl->mg_c[c]);
  for (const void* q : {(const void*)pl->mg_u, (const void*)pl->mg_t, (const void*)pl->mg_f, (const void*)pl->mg_Fc,
                        (const void*)pl->mg_Uc, (const void*)pl->mg_T1c, (const void*)pl->mg_T2c,
                        (const void*)pl->mg_twc, (const void*)pl->mg_eigc, (const void*)pl->mg_part,
                        (const void*)pl->mg_ctl, (const void*)pl->mg_scal, (const void*)pl->scal})
    put((uint64_t)(uintptr_t)q);
}
}  // namespace

void mg_graphs_clear(kfbi_plan* pl) {
  for (int i = 0; i < pl->mg_sg_n; ++i) {
    if (pl->mg_sg[i].e) (void)hipGraphExecDestroy(pl->mg_sg[i].e);
    if (pl->mg_sg[i].g) (void)hipGraphDestroy(pl->mg_sg[i].g);
  }
  pl->mg_sg_n = 0;
}

// A solve is a few hundred short kernels whose launches cost more than
// their work on small grids: it goes out as one graph, captured on first
// use.  Inside a capture of the caller's (or with the tracing events of
// profile modes 2 and 3) the kernels are enqueued as they are.
void mg_solve(kfbi_plan* pl, const double* F, double* v) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const hipStream_t st = pl->stream;
  // (the default streams cannot be captured)
  if (pl->mg_graphs_off || pl->prof_on >= 2 || st == nullptr || st == hipStreamLegacy || st == hipStreamPerThread ||
      hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
    solve_enqueue(pl, F, v);
    return;
  }
  uint64_t key[48];
  config_key(pl, key);
  if (memcmp(key, pl->mg_sg_key, sizeof(key)) != 0) {
    mg_graphs_clear(pl);
    memcpy(pl->mg_sg_key, key, sizeof(key));
  }
  const int cap = pl->mg_run_cap > 0 ? pl->mg_run_cap : pl->mg_maxit;
  const int guess = pl->mg_guess ? 1 : 0;
  for (int i = 0; i < pl->mg_sg_n; ++i) {
    const kfbi_plan::MgSolveGraph& e = pl->mg_sg[i];
    if (e.F == F && e.v == v && e.gctl == pl->ctl_active && e.cap == cap && e.guess == guess && e.eps == pl->mg_eps) {
      if (hipGraphLaunch(e.e, pl->stream) == hipSuccess) return;
      (void)hipGetLastError();
      pl->mg_graphs_off = true;
      solve_enqueue(pl, F, v);
      return;
    }
  }
  // capture exclusive of other threads' set-up and allocations; a thread
  // that cannot have the lock now enqueues the kernels instead
  std::unique_lock<std::shared_mutex> lock(kfbi_capture_mutex, std::try_to_lock);
  if (!lock.owns_lock()) {
    solve_enqueue(pl, F, v);
    return;
  }
  if (pl->mg_sg_n == KFBI_MG_GRAPHS) mg_graphs_clear(pl);
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
  bool ok = hipStreamBeginCapture(pl->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    solve_enqueue(pl, F, v);
    ok = hipStreamEndCapture(pl->stream, &g) == hipSuccess && g;
  }
  ok = ok && hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess;
  ok = ok && hipGraphLaunch(ex, pl->stream) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    if (ex) (void)hipGraphExecDestroy(ex);
    if (g) (void)hipGraphDestroy(g);
    pl->mg_graphs_off = true;
    solve_enqueue(pl, F, v);
    return;
  }
  pl->mg_sg[pl->mg_sg_n++] = kfbi_plan::MgSolveGraph{F, v, pl->ctl_active, cap, guess, pl->mg_eps, g, ex};
}

// 1 + 64 slots, and at most 2 GiB
kfbi_status mg_store_reserve(kfbi_plan* pl) {
  const int64_t n = pl->g.n_nodes;
  if (pl->ustore && pl->ustore_n == n) return KFBI_OK;
  if (pl->ustore) (void)hipFree(pl->ustore);
  pl->ustore = nullptr;
  pl->ustore_slots = 0;
  pl->ustore_n = 0;
  int64_t slots = ((int64_t)2 << 30) / (8 * n);
  if (slots > 65) slots = 65;
  if (slots < 2) return KFBI_OK;         // too large a grid: solves run without the store
  if (hipMalloc((void**)&pl->ustore, sizeof(double) * n * slots) != hipSuccess) {
    (void)hipGetLastError();
    pl->ustore = nullptr;
    return KFBI_OK;                      // the store is an optimisation: go without it
  }
  pl->ustore_slots = (int)slots;
  pl->ustore_n = n;
  return KFBI_OK;
}

void mg_store_solution(kfbi_plan* pl, const double* v) {
  if (!pl->ustore) return;
  hipLaunchKernelGGL(k_ustore, dim3(gsblk(pl->ustore_n)), dim3(MG_BLOCK), 0, pl->stream, pl->ctl_active,
                     pl->ustore_n, pl->ustore_slots, v, pl->ustore);
}

void mg_guess_from_store(kfbi_plan* pl, int k, int use_x0, const double* y, double* v) {
  hipLaunchKernelGGL(k_ucombine, dim3(gsblk(pl->ustore_n)), dim3(MG_BLOCK), 0, pl->stream, pl->ustore_n, k,
                     use_x0, y, (const double*)pl->ustore, v);
}

void mg_sum(kfbi_plan* pl, const double* a, const double* b, double* out) {
  hipLaunchKernelGGL(k_usum, dim3(gsblk(pl->g.n_nodes)), dim3(MG_BLOCK), 0, pl->stream, pl->g.n_nodes, a, b, out);
}

void vec_diff(kfbi_plan* pl, int64_t n, const double* a, const double* b, double* out) {
  if (n > 0) hipLaunchKernelGGL(k_udiff, dim3(gsblk(n)), dim3(MG_BLOCK), 0, pl->stream, n, a, b, out);
}

void grid_zero(kfbi_plan* pl, double* v) {
  hipLaunchKernelGGL(k_uzero, dim3(gsblk(pl->g.n_nodes)), dim3(MG_BLOCK), 0, pl->stream, pl->g.n_nodes, v);
}

void mg_matvec_rhs(kfbi_plan* pl) {
  if (pl->n_irr == 0) return;
  hipLaunchKernelGGL(k_scatter, dim3(nblk(pl->n_irr)), dim3(MG_BLOCK), 0, pl->stream, pl->ctl_active, pl->n_irr,
                     pl->maxpairs, pl->irr, pl->PA, pl->PE1, pl->PE2, pl->Cv, pl->Fmg);
}
