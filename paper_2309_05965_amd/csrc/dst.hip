// Step S3 -- box solve A_h v = F with homogeneous Dirichlet data.
//
// Paper: Alg. 1 Step 3.3 solves the corrected finite-difference system "with
// FFT"; Sec. 5.2 gives the operators (eqs. 9p-cds, 27p-cds).  With
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
// sequence of length M = 2N, runs radix-2 FFTs in LDS, and unpacks both
// sine transforms from the result (Re Z_k = 2 S_B(k), Im Z_k = -2 S_A(k)).
// The last axis is fused: forward DST, spectral divide and inverse DST in
// LDS, so 2D takes 3 passes and 3D 5 passes of 16 B per node.
#include <math.h>

#include <vector>

#include "kfbi_internal.h"

namespace {

constexpr int LDS_COMPLEX = 4096;   // complex slots for the FFT working set (64 KiB)

struct DstArgs {
  GridDesc g;
  int ax;          // transform axis
  int mode;        // 0: DST; 1: DST, divide by lambda and scale, DST
  int TL;          // lines per tile (even)
  int M, logM;     // FFT length 2N
  int tiles_u;     // tiles along the tile axis
  const double* in;
  double* out;
  const double2* tw;   // exp(-2 pi i m / M), m < M/2
  const double* eig1;  // s_k, k = 0..N
  double scale;        // (2/N)^d
};

__device__ __forceinline__ unsigned bitrev(unsigned x, int bits) { return __brev(x) >> (32 - bits); }

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// In-place radix-2 DIT FFTs of nf sequences of length M held in bit-reversed
// order in buf[f * M + i].
__device__ void fft_lds(double2* buf, const double2* tw, int nf, int M, int logM) {
  const int half_total = nf * (M / 2);
  for (int s = 1; s <= logM; ++s) {
    const int half = 1 << (s - 1);
    const int tstride = M / (2 * half);
    for (int b = threadIdx.x; b < half_total; b += blockDim.x) {
      int f = b / (M / 2);
      int i = b % (M / 2);
      int grp = i / half, pos = i % half;
      int i0 = f * M + grp * 2 * half + pos;
      int i1 = i0 + half;
      double2 w = tw[pos * tstride];
      double2 t = cmul(w, buf[i1]);
      double2 u = buf[i0];
      buf[i0] = make_double2(u.x + t.x, u.y + t.y);
      buf[i1] = make_double2(u.x - t.x, u.y - t.y);
    }
    __syncthreads();
  }
}

// coordinate of line l of the tile and element j (1..N-1) along the axis
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

__global__ void __launch_bounds__(KFBI_BLOCK) k_dst(DstArgs a) {
  extern __shared__ double2 lds[];
  double2* buf = lds;                               // [nf][M]
  double2* tw = lds + (a.TL / 2) * a.M;             // [M/2]
  const GridDesc& g = a.g;
  const int N = g.N, M = a.M, TL = a.TL, nf = TL / 2;
  const int tile = blockIdx.x % a.tiles_u;
  const int w = blockIdx.x / a.tiles_u + 1;         // remaining interior coordinate (3D)
  const int u0 = 1 + tile * TL;                     // first tile coordinate
  for (int m = threadIdx.x; m < M / 2; m += blockDim.x) tw[m] = a.tw[m];
  // zero the working set (positions 0 and N of every sequence stay zero)
  for (int i = threadIdx.x; i < nf * M; i += blockDim.x) buf[i] = make_double2(0.0, 0.0);
  __syncthreads();
  const int nl = N - 1;
  const int total = TL * nl;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    int l, j;
    if (a.ax == 0) {
      j = idx % nl + 1;
      l = idx / nl;
    } else {
      l = idx % TL;
      j = idx / TL + 1;
    }
    int u = u0 + l;
    double x = u <= N - 1 ? a.in[elem_addr(a, u, w, j)] : 0.0;
    int f = l >> 1;
    unsigned p1 = bitrev((unsigned)j, a.logM), p2 = bitrev((unsigned)(M - j), a.logM);
    if (l & 1) {
      buf[f * M + p1].y = x;
      buf[f * M + p2].y = -x;
    } else {
      buf[f * M + p1].x = x;
      buf[f * M + p2].x = -x;
    }
  }
  __syncthreads();
  fft_lds(buf, tw, nf, M, a.logM);
  if (a.mode == 1) {
    // unpack, divide by lambda and scale; the scaled coefficients are
    // stashed in the unused upper half of each sequence, then re-placed as
    // new odd sequences in bit-reversed order for the inverse transform
    for (int idx = threadIdx.x; idx < nf * nl; idx += blockDim.x) {
      int f = idx / nl, k = idx % nl + 1;
      double2 Z = buf[f * M + k];
      // S_A = -Im/2 (even line), S_B = Re/2 (odd line)
      double SA = -0.5 * Z.y, SB = 0.5 * Z.x;
      int uA = u0 + 2 * f, uB = uA + 1;
      // mode indices of the already transformed axes are the line coordinates
      double s_ax = a.eig1[k];
      double lamA, lamB;
      {
        double sA[3], sB[3];
        int ua = a.ax == 0 ? 1 : 0;
        for (int t = 0; t < 3; ++t) sA[t] = sB[t] = 0.0;
        sA[a.ax] = s_ax;
        sB[a.ax] = s_ax;
        sA[ua] = a.eig1[uA <= N - 1 ? uA : 1];
        sB[ua] = a.eig1[uB <= N - 1 ? uB : 1];
        if (g.d == 3) {
          int wa = 3 - a.ax - ua;
          sA[wa] = a.eig1[w];
          sB[wa] = a.eig1[w];
        }
        double h2 = g.h * g.h;
        double lapA = 0.0, lapB = 0.0, prA = 0.0, prB = 0.0;
        for (int t = 0; t < g.d; ++t) {
          lapA += sA[t];
          lapB += sB[t];
          for (int t2 = t + 1; t2 < g.d; ++t2) {
            prA += sA[t] * sA[t2];
            prB += sB[t] * sB[t2];
          }
        }
        if (g.order == 2) {
          lamA = lapA - g.kappa;
          lamB = lapB - g.kappa;
        } else {
          lamA = lapA + h2 / 6.0 * prA;
          lamB = lapB + h2 / 6.0 * prB;
          if (g.d == 3) {
            lamA += h2 * h2 / 48.0 * sA[0] * sA[1] * sA[2];
            lamB += h2 * h2 / 48.0 * sB[0] * sB[1] * sB[2];
          }
          lamA -= g.kappa * (1.0 + h2 / 12.0 * lapA);
          lamB -= g.kappa * (1.0 + h2 / 12.0 * lapB);
        }
      }
      // stash the scaled coefficients in the (unused) slot M - k
      buf[f * M + (M - k)] = make_double2(a.scale * SA / lamA, a.scale * SB / lamB);
    }
    __syncthreads();
    // move stashed values into registers per thread, zero, and re-place
    for (int f0 = 0; f0 < nf; ++f0) {
      // each pass handles one sequence to keep the register footprint small
      double2 keep[8];
      int cnt = 0;
      for (int k = threadIdx.x + 1; k <= nl && cnt < 8; k += blockDim.x) keep[cnt++] = buf[f0 * M + (M - k)];
      __syncthreads();
      for (int i = threadIdx.x; i < M; i += blockDim.x) buf[f0 * M + i] = make_double2(0.0, 0.0);
      __syncthreads();
      cnt = 0;
      for (int k = threadIdx.x + 1; k <= nl && cnt < 8; k += blockDim.x) {
        double2 v = keep[cnt++];
        unsigned p1 = bitrev((unsigned)k, a.logM), p2 = bitrev((unsigned)(M - k), a.logM);
        buf[f0 * M + p1] = make_double2(v.x, v.y);
        buf[f0 * M + p2] = make_double2(-v.x, -v.y);
      }
      __syncthreads();
    }
    fft_lds(buf, tw, nf, M, a.logM);
  }
  // unpack and store
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    int l, k;
    if (a.ax == 0) {
      k = idx % nl + 1;
      l = idx / nl;
    } else {
      l = idx % TL;
      k = idx / TL + 1;
    }
    int u = u0 + l;
    if (u > N - 1) continue;
    double2 Z = buf[(l >> 1) * M + k];
    double v = (l & 1) ? 0.5 * Z.x : -0.5 * Z.y;
    a.out[elem_addr(a, u, w, k)] = v;
  }
}

// lines per tile: (TL/2) sequences of M complex values plus M/2 twiddles
// within LDS_COMPLEX complex slots (64 KiB)
int tile_lines(int M) {
  int nf = (LDS_COMPLEX - M / 2) / M;
  if (nf > 16) nf = 16;
  if (nf < 1) nf = 1;
  return 2 * nf;
}

void launch_pass(kfbi_plan* pl, int ax, int mode, const double* in, double* out) {
  DstArgs a;
  a.g = pl->g;
  a.ax = ax;
  a.mode = mode;
  a.M = 2 * pl->g.N;
  a.logM = 0;
  while ((1 << a.logM) < a.M) ++a.logM;
  int nl = pl->g.N - 1;
  // enough work groups to fill 256 CUs: aim at >= 1024 tiles, at least one
  // FFT (two lines) per tile, at most what fits the LDS budget
  int64_t lines = pl->g.d == 3 ? (int64_t)nl * nl : nl;
  int64_t tl = 2 * (lines / 2048);
  if (tl < 2) tl = 2;
  if (tl > tile_lines(a.M)) tl = tile_lines(a.M);
  a.TL = (int)tl;
  a.tiles_u = (nl + a.TL - 1) / a.TL;
  a.in = in;
  a.out = out;
  a.tw = (const double2*)pl->tw;
  a.eig1 = pl->eig1;
  a.scale = 1.0;
  for (int t = 0; t < pl->g.d; ++t) a.scale *= 2.0 / pl->g.N;
  unsigned blocks = (unsigned)a.tiles_u * (pl->g.d == 3 ? nl : 1);
  size_t lds = sizeof(double2) * ((size_t)(a.TL / 2) * a.M + a.M / 2);
  hipLaunchKernelGGL(k_dst, dim3(blocks), dim3(KFBI_BLOCK), lds, pl->stream, a);
}

}  // namespace

kfbi_status dst_init(kfbi_plan* pl) {
  int N = pl->g.N, M = 2 * N;
  std::vector<double> tw((size_t)M), eig((size_t)N + 1);
  for (int m = 0; m < M / 2; ++m) {
    double ang = -2.0 * M_PI * (double)m / (double)M;
    tw[2 * m] = cos(ang);
    tw[2 * m + 1] = sin(ang);
  }
  for (int k = 0; k <= N; ++k) {
    double sn = sin((double)k * M_PI / (2.0 * N));
    eig[k] = -4.0 / (pl->g.h * pl->g.h) * sn * sn;
  }
  HIPCHK(hipMemcpy(pl->tw, tw.data(), sizeof(double) * M, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(pl->eig1, eig.data(), sizeof(double) * (N + 1), hipMemcpyHostToDevice));
  int lds = (int)(sizeof(double2) * ((size_t)(tile_lines(M) / 2) * M + M / 2));
  if (lds > 65536) {
    kfbi_set_error("box solver LDS footprint too large (N = %d)", N);
    return KFBI_E_INVALID;
  }
  return KFBI_OK;
}

void dst_solve(kfbi_plan* pl, const double* F, double* v) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (pl->prof_on && pl->prof_ev) {
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
