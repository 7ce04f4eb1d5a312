// Steps S10 / S11 -- learned initial density for GMRES (Alg. 1 Step 2).
//
// A small MLP maps features of 1024 interface samples (position, outward
// normal, mean curvature, g1, g2) to the density at the samples; a
// least-squares fit of real spherical harmonics (degree <= 8, body-frame
// direction of the ellipsoid) carries it to the DOFs.  Training minimises
// the mean squared error against densities the solver itself produced,
// with hand-written bf16 MFMA GEMMs (v_mfma_f32_16x16x32_bf16, fp32
// accumulation) for the forward and backward passes and Adam on fp32
// master weights.
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "kfbi_internal.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

// ---------------------------------------------------------------- bf16
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);          // round to nearest, ties to even
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------- GEMM
// C[M x N] = op(A) op(B), bf16 operands, fp32 accumulation.
//   A: AT = false -> stored [M x K] (row stride lda), AT = true -> [K x M]
//   B: BT = false -> stored [K x N] (row stride ldb), BT = true -> [N x K]
// Epilogue per element (row r, column c): v = acc (+ bias[c]); if mask,
// v = z[r, c] > 0 ? v : 0 (ReLU derivative of a stored pre-activation);
// written to Cf (fp32) as is and to Cb (bf16) after max(v, 0) when relu_b,
// row stride ldc.  Workgroup tile 64 x 64 (four wavefronts of 32 x 32, each
// 2 x 2 MFMA 16 x 16 tiles), K step 32.  Each thread moves eight
// consecutive bf16 of each operand tile per step, as one 16-byte load when
// the rows are 16-byte aligned (vec) and the eight are in range; the next
// step's loads are issued before the current step's MFMAs and land in the
// other of two LDS buffers, so one barrier per step separates them.
constexpr int GBM = 64, GBN = 64, GBK = 32, GPAD = 8;

struct GemmArgs {
  int M, N, K, lda, ldb, ldc;
  const uint16_t* A;
  const uint16_t* B;
  const float* bias;
  const float* z;       // mask source (ldc stride) or null
  int relu_b;           // bf16 output is max(v, 0)
  float* Cf;
  uint16_t* Cb;
  int vec_a, vec_b;     // rows 16-byte aligned: eight-element chunks as one load
  int kchunk;           // split K: work group z multiplies K range [z kchunk, (z + 1) kchunk)
  int64_t zstride;      // and writes its partial product to Cf + z zstride (no epilogue)
};

union Chunk8 {
  uint4 v;
  uint16_t h[8];
};

// eight consecutive elements p[0..7] of a row, n of them in range (the rest 0)
__device__ __forceinline__ Chunk8 load8(const uint16_t* p, int n, bool vec) {
  Chunk8 c;
  if (vec && n >= 8) {
    c.v = *reinterpret_cast<const uint4*>(p);
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) c.h[i] = i < n ? p[i] : (uint16_t)0;
  }
  return c;
}

template <bool AT, bool BT>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t As[2][GBM][GBK + GPAD];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][GBN][GBK + GPAD];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  // this thread's chunk of the A and B tiles: non-transposed, row r and
  // columns kc..kc+7 of K; transposed, K row kk and columns c8..c8+7
  const int r = t >> 2, kc = (t & 3) * 8, kk = t >> 3, c8 = (t & 7) * 8;
  const int kbeg = blockIdx.z * g.kchunk;
  const int kend = kbeg + g.kchunk < g.K ? kbeg + g.kchunk : g.K;
  auto load_a = [&](int k0) -> Chunk8 {
    if (!AT) {
      const int gm = m0 + r, gk = k0 + kc;
      const int n = gm < g.M ? kend - gk : 0;
      return load8(g.A + (int64_t)gm * g.lda + gk, n < 8 ? (n < 0 ? 0 : n) : 8, g.vec_a);
    }
    const int gk = k0 + kk, gm = m0 + c8;
    const int n = gk < kend ? g.M - gm : 0;
    return load8(g.A + (int64_t)gk * g.lda + gm, n < 8 ? (n < 0 ? 0 : n) : 8, g.vec_a);
  };
  auto load_b = [&](int k0) -> Chunk8 {
    if (BT) {
      const int gn = n0 + r, gk = k0 + kc;
      const int n = gn < g.N ? kend - gk : 0;
      return load8(g.B + (int64_t)gn * g.ldb + gk, n < 8 ? (n < 0 ? 0 : n) : 8, g.vec_b);
    }
    const int gk = k0 + kk, gn = n0 + c8;
    const int n = gk < kend ? g.N - gn : 0;
    return load8(g.B + (int64_t)gk * g.ldb + gn, n < 8 ? (n < 0 ? 0 : n) : 8, g.vec_b);
  };
  auto store = [&](int buf, const Chunk8& ca, const Chunk8& cb) {
    if (!AT) {
      *reinterpret_cast<uint4*>(&As[buf][r][kc]) = ca.v;
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) As[buf][c8 + i][kk] = ca.h[i];
    }
    if (BT) {
      *reinterpret_cast<uint4*>(&Bs[buf][r][kc]) = cb.v;
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) Bs[buf][c8 + i][kk] = cb.h[i];
    }
  };
  f32x4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
  const int nk = kend > kbeg ? (kend - kbeg + GBK - 1) / GBK : 0;
  {
    const Chunk8 ca = load_a(kbeg), cb = load_b(kbeg);
    store(0, ca, cb);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    Chunk8 na, nbv;
    const bool more = kt + 1 < nk;
    if (more) {
      na = load_a(kbeg + (kt + 1) * GBK);
      nbv = load_b(kbeg + (kt + 1) * GBK);
    }
    const int ko = (lane >> 4) * 8;
    bf16x8 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8*>(&As[cur][wr + 16 * i + (lane & 15)][ko]);
#pragma unroll
    for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const bf16x8*>(&Bs[cur][wc + 16 * j + (lane & 15)][ko]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    if (more) store(cur ^ 1, na, nbv);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = m0 + wr + 16 * i + 4 * (lane >> 4) + q;
        const int col = n0 + wc + 16 * j + (lane & 15);
        if (row >= g.M || col >= g.N) continue;
        float v = acc[i][j][q];
        const int64_t o = (int64_t)row * g.ldc + col;
        if (gridDim.z > 1) {
          g.Cf[blockIdx.z * g.zstride + o] = v;
          continue;
        }
        if (g.bias) v += g.bias[col];
        if (g.z) v = g.z[o] > 0.f ? v : 0.f;
        if (g.Cf) g.Cf[o] = v;
        if (g.Cb) g.Cb[o] = to_bf16(g.relu_b && v < 0.f ? 0.f : v);
      }
}

// ---------------------------------------------------------------- few-row products
// For a batch of at most GV_BMAX rows the 64 x 64 MFMA tiles leave almost
// the whole chip idle (one tile row, K looped serially), so the forward pass
// splits K instead: workgroup (x, y) multiplies the rows by a GV_KC-row
// slab y of W for 256 columns x, fp32 accumulation of bf16 products, and
// writes one partial per (row, column, slab); a second kernel sums the
// slabs in a fixed order and applies the GEMM epilogue.  W row-major
// [K x N], N and the row stride multiples of 8 (16-byte loads).
constexpr int GV_BMAX = 8, GV_COLS = 256, GV_KC = 64;

__global__ void __launch_bounds__(256) k_gemv_part(int B, int N, int K, const uint16_t* A, int lda,
                                                   const uint16_t* W, int ldw, float* part) {
  __shared__ float red[8][GV_BMAX][GV_COLS];
  const int t = threadIdx.x, cg = t & 31, rg = t >> 5;
  const int c0 = blockIdx.x * GV_COLS + cg * 8;
  const int k0 = blockIdx.y * GV_KC;
  const int k1 = K - k0 < GV_KC ? K : k0 + GV_KC;
  float acc[GV_BMAX][8];
#pragma unroll
  for (int b = 0; b < GV_BMAX; ++b)
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[b][i] = 0.f;
  if (c0 < N) {
    for (int k = k0 + rg; k < k1; k += 8) {
      const uint4 w = *reinterpret_cast<const uint4*>(W + (int64_t)k * ldw + c0);
      const uint32_t wu[4] = {w.x, w.y, w.z, w.w};
      float wf[8];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        wf[2 * i] = __uint_as_float(wu[i] << 16);
        wf[2 * i + 1] = __uint_as_float(wu[i] & 0xffff0000u);
      }
#pragma unroll
      for (int b = 0; b < GV_BMAX; ++b) {
        if (b < B) {
          const float a = from_bf16(A[(int64_t)b * lda + k]);
#pragma unroll
          for (int i = 0; i < 8; ++i) acc[b][i] = fmaf(a, wf[i], acc[b][i]);
        }
      }
    }
  }
#pragma unroll
  for (int b = 0; b < GV_BMAX; ++b)
#pragma unroll
    for (int i = 0; i < 8; ++i) red[rg][b][cg * 8 + i] = acc[b][i];
  __syncthreads();
  const int nch = gridDim.y;
  for (int e = t; e < B * GV_COLS; e += 256) {
    const int b = e / GV_COLS, c = e % GV_COLS;
    const int col = blockIdx.x * GV_COLS + c;
    if (col >= N) continue;
    float s = 0.f;
#pragma unroll
    for (int r = 0; r < 8; ++r) s += red[r][b][c];
    part[((int64_t)b * N + col) * nch + blockIdx.y] = s;
  }
}

// out[o] (o = row * N + column) = sum of the slabs (one wavefront per
// output, fixed order) + bias; epilogue as in k_gemm (row stride N)
__global__ void __launch_bounds__(256) k_gemv_sum(int BN, int N, int nch, const float* part, const float* bias,
                                                  int relu_b, float* Cf, uint16_t* Cb) {
  const int o = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (o >= BN) return;
  const float* p = part + (int64_t)o * nch;
  float s = 0.f;
  for (int q = lane; q < nch; q += 64) s += p[q];
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
  if (lane == 0) {
    const float v = bias ? s + bias[o % N] : s;
    if (Cf) Cf[o] = v;
    if (Cb) Cb[o] = to_bf16(relu_b && v < 0.f ? 0.f : v);
  }
}

// ---------------------------------------------------------------- elementwise
__global__ void k_to_bf16(int64_t n, const float* x, uint16_t* y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = to_bf16(x[i]);
}

// output gradient of L = mean (o - y)^2: dz = 2 (o - y) / n (fp32 and bf16)
// and per-block sums of (o - y)^2
__global__ void __launch_bounds__(256) k_mse(int64_t n, const float* o, const float* y, float* dz,
                                             uint16_t* dzb, double* part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float d = o[i] - y[i];
    acc += (double)d * (double)d;
    const float gz = 2.f * d / (float)n;
    dz[i] = gz;
    dzb[i] = to_bf16(gz);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < (unsigned)s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_loss_final(int nb, int64_t n, const double* part, float* loss) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < nb; ++i) s += part[i];
  *loss = (float)(s / (double)n);
}

// db[c] = sum over rows of dz[r, c], in a fixed order: work group (x, y)
// sums 64 columns over row slab y (4 row phases of 64 threads, then the
// phases in order) into part[y][c]; k_colsum_final adds the slabs in order
constexpr int CS_SLABS = 16;
constexpr int SK_MAX = 16;   // split-K partials at most
__global__ void __launch_bounds__(256) k_colsum(int rows, int cols, const float* dz, float* part) {
  __shared__ float sh[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), ph = threadIdx.x >> 6;
  const int per = (rows + CS_SLABS - 1) / CS_SLABS;
  const int r0 = blockIdx.y * per, r1 = r0 + per < rows ? r0 + per : rows;
  float s = 0.f;
  if (c < cols)
    for (int r = r0 + ph; r < r1; r += 4) s += dz[(int64_t)r * cols + c];
  sh[ph][threadIdx.x & 63] = s;
  __syncthreads();
  if (ph == 0 && c < cols)
    part[(int64_t)blockIdx.y * cols + c] = ((sh[0][threadIdx.x] + sh[1][threadIdx.x]) + sh[2][threadIdx.x]) +
                                           sh[3][threadIdx.x];
}

__global__ void k_colsum_final(int cols, int slabs, const float* part, float* db) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int y = 0; y < slabs; ++y) s += part[(int64_t)y * cols + c];
  db[c] = s;
}

// C = sum over the split-K partials, in order
__global__ void k_splitk_sum(int64_t n, int S, int64_t stride, const float* part, float* C) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int z = 0; z < S; ++z) s += part[z * stride + i];
  C[i] = s;
}

// Linear head (the density is linear in the jump coefficients): the last
// layer's output row z of example b holds nb basis vectors of K entries,
// y[b, k] = sum_j C[b, j] z[b, j K + k] (fp32).
__global__ void k_lin_head_fwd(int B, int nb, int K, const float* C, const float* Z, float* Y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)B * K) return;
  const int b = (int)(t / K), k = (int)(t % K);
  const float* z = Z + (int64_t)b * nb * K;
  float s = 0.f;
  for (int j = 0; j < nb; ++j) s += C[(int64_t)b * nb + j] * z[(int64_t)j * K + k];
  Y[t] = s;
}

// gradient of the head: dz[b, j K + k] = C[b, j] dy[b, k] (fp32 and bf16)
__global__ void k_lin_head_bwd(int B, int nb, int K, const float* C, const float* dy, float* dz, uint16_t* dzb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)B * nb * K) return;
  const int64_t b = t / ((int64_t)nb * K);
  const int r = (int)(t % ((int64_t)nb * K));
  const int j = r / K, k = r % K;
  const float g = C[b * nb + j] * dy[b * K + k];
  dz[t] = g;
  dzb[t] = to_bf16(g);
}

// the prediction's head in FP64 output: coef[k] = scale sum_{m,t} c[t 8 + m]
// z[(m 4 + t) K + k], z the 8 rows (one per Fourier mode m) of 4 basis
// vectors each (t: a_1m, a_2m, b_1m, b_2m; c in the packed order a_1[8],
// a_2[8], b_1[8], b_2[8])
__global__ void k_lin_head_coef(int K, const double* c, const float* z, double scale, double* coef) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  double s = 0.0;
  for (int m = 0; m < 8; ++m)
    for (int t = 0; t < 4; ++t) s += c[t * 8 + m] * (double)z[(int64_t)(m * 4 + t) * K + k];
  coef[k] = scale * s;
}

// network input of the linear-head start: one row per ellipsoid and Fourier
// mode m (k_m = (pi/2)(m & 1, (m >> 1) & 1, (m >> 2) & 1)): the semi-axes
// centred and scaled from U(0.3, 0.7) to [-1, 1], the mode's wave vector in
// the scaled body frame diag(a) Q^T k_m (cos(k_m . x) = cos(kappa . s) on
// the ellipsoid x = Q diag(a) s), and the nine entries of Q
constexpr int GEOM_IN = 15;
__global__ void k_geom_input(int P, const double* geom, float* X) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P * 8) return;
  const int p = t >> 3, m = t & 7;
  const double* G = geom + 15 * (int64_t)p;
  const double* a = G + 3;
  const double* Q = G + 6;
  const double h = 1.5707963267948966;
  const double k[3] = {(m & 1) * h, ((m >> 1) & 1) * h, ((m >> 2) & 1) * h};
  float* x = X + (int64_t)t * GEOM_IN;
  for (int i = 0; i < 3; ++i) {
    x[i] = (float)((a[i] - 0.5) / 0.2);
    x[3 + i] = (float)(a[i] * (Q[i] * k[0] + Q[3 + i] * k[1] + Q[6 + i] * k[2]));
  }
  for (int i = 0; i < 9; ++i) x[6 + i] = (float)Q[i];
}

// Adam on fp32 masters; bf16 copies of the weight matrices are refreshed
struct AdamArgs {
  int64_t n;
  float lr, b1, b2, eps, c1, c2;   // c1 = 1 - b1^t, c2 = 1 - b2^t
  float *w, *m, *v;
  const float* g;
  const int64_t* bf_index;         // position in the bf16 copy (-1 for biases)
  uint16_t* wb;
};

__global__ void k_adam(AdamArgs a) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const float g = a.g[i];
  const float m = a.b1 * a.m[i] + (1.f - a.b1) * g;
  const float v = a.b2 * a.v[i] + (1.f - a.b2) * g * g;
  a.m[i] = m;
  a.v[i] = v;
  const float w = a.w[i] - a.lr * (m / a.c1) / (sqrtf(v / a.c2) + a.eps);
  a.w[i] = w;
  const int64_t j = a.bf_index[i];
  if (j >= 0) a.wb[j] = to_bf16(w);
}

__global__ void k_refresh_bf16(int64_t n, const float* w, const int64_t* bf_index, uint16_t* wb) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t j = bf_index[i];
  if (j >= 0) wb[j] = to_bf16(w[i]);
}

// data augmentation by the linearity of the density in the jump data: the
// g1, g2 features (columns 7, 8 of every sample) and the target row of
// example r are multiplied by alpha[r]
__global__ void k_scale_jumps(int B, int ns, int nout, const float* alpha, float* X, float* Y) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nx = (int64_t)B * ns * 2;
  if (t < nx) {
    const int64_t r = t / (2 * ns), q = t % (2 * ns);
    X[r * ns * 9 + (q >> 1) * 9 + 7 + (q & 1)] *= alpha[r];
  } else if (t < nx + (int64_t)B * nout) {
    const int64_t u = t - nx;
    Y[u] *= alpha[u / nout];
  }
}

// ---------------------------------------------------------------- features
// geometry per problem: c (3), semi-axes a (3), Q row-major (9); jumps per
// problem: a[j][m] (16) then b[j][m] (16), j = 0 (g1), 1 (g2), m < 8 with
// k_m = (pi/2) (m & 1, (m >> 1) & 1, (m >> 2) & 1)
__device__ __forceinline__ void jump_at(const double* J, const double* x, double& g1, double& g2) {
  g1 = 0.0;
  g2 = 0.0;
  for (int m = 0; m < 8; ++m) {
    const double ph = 0.5 * M_PI * ((double)(m & 1) * x[0] + (double)((m >> 1) & 1) * x[1] + (double)((m >> 2) & 1) * x[2]);
    const double cp = cos(ph), sp = sin(ph);
    g1 += J[m] * cp + J[16 + m] * sp;
    g2 += J[8 + m] * cp + J[24 + m] * sp;
  }
}

__global__ void k_features(int P, int ns, const double* geom, const double* jumps, const double* S, float* X) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)P * ns) return;
  const int p = (int)(t / ns), i = (int)(t % ns);
  const double* G = geom + 15 * (int64_t)p;
  const double* a = G + 3;
  const double* Q = G + 6;
  double Xb[3], x[3], gb[3], n[3];
  for (int k = 0; k < 3; ++k) Xb[k] = a[k] * S[3 * (int64_t)i + k];
  for (int r = 0; r < 3; ++r) x[r] = G[r] + Q[3 * r] * Xb[0] + Q[3 * r + 1] * Xb[1] + Q[3 * r + 2] * Xb[2];
  double hs = 0.0, ng2 = 0.0, ghg = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double hk = 2.0 / (a[k] * a[k]);
    gb[k] = hk * Xb[k];
    hs += hk;
    ng2 += gb[k] * gb[k];
    ghg += gb[k] * gb[k] * hk;
  }
  const double ng = sqrt(ng2);
  for (int r = 0; r < 3; ++r) n[r] = (Q[3 * r] * gb[0] + Q[3 * r + 1] * gb[1] + Q[3 * r + 2] * gb[2]) / ng;
  const double kappa = (ng2 * hs - ghg) / (2.0 * ng2 * ng);
  double g1, g2;
  jump_at(jumps + 32 * (int64_t)p, x, g1, g2);
  float* o = X + (int64_t)p * ns * 9 + (int64_t)i * 9;
  o[0] = (float)x[0];
  o[1] = (float)x[1];
  o[2] = (float)x[2];
  o[3] = (float)n[0];
  o[4] = (float)n[1];
  o[5] = (float)n[2];
  o[6] = (float)kappa;
  o[7] = (float)g1;
  o[8] = (float)g2;
}

// ---------------------------------------------------------------- spherical harmonics
constexpr int SH_L = 8;
constexpr int SH_N = (SH_L + 1) * (SH_L + 1);

// real orthonormal spherical harmonics (no Condon-Shortley phase) of the
// direction d (not necessarily unit), index l^2 + l + m
__device__ void real_sh(const double* d, double* Y) {
  const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  const double ct = d[2] / r;
  const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
  double cphi = 1.0, sphi = 0.0;
  const double rho = sqrt(d[0] * d[0] + d[1] * d[1]);
  if (rho > 0.0) {
    cphi = d[0] / rho;
    sphi = d[1] / rho;
  }
  double cm[SH_L + 1], sm[SH_L + 1];
  cm[0] = 1.0;
  sm[0] = 0.0;
  for (int m = 1; m <= SH_L; ++m) {
    cm[m] = cm[m - 1] * cphi - sm[m - 1] * sphi;
    sm[m] = sm[m - 1] * cphi + cm[m - 1] * sphi;
  }
  // normalised associated Legendre values Q_l^m = N_lm P_l^m(ct), m <= l
  double qmm = 0.5 / sqrt(M_PI);          // Q_0^0
  for (int m = 0; m <= SH_L; ++m) {
    if (m > 0) qmm = qmm * st * sqrt((2.0 * m + 1.0) / (2.0 * m));
    double q2 = 0.0, q1 = qmm;
    for (int l = m; l <= SH_L; ++l) {
      double q;
      if (l == m) {
        q = qmm;
      } else if (l == m + 1) {
        q = ct * sqrt(2.0 * m + 3.0) * qmm;
      } else {
        const double al = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
        const double bl = sqrt((((double)(l - 1) * (l - 1)) - (double)m * m) / (4.0 * (l - 1) * (l - 1) - 1.0));
        q = al * (ct * q1 - bl * q2);
      }
      if (l > m) {
        q2 = q1;
        q1 = q;
      }
      if (m == 0) {
        Y[l * l + l] = q;
      } else {
        Y[l * l + l + m] = sqrt(2.0) * q * cm[m];
        Y[l * l + l - m] = sqrt(2.0) * q * sm[m];
      }
    }
  }
}

// body-frame direction diag(1/a) Q^T (x - c) of a point x
__device__ __forceinline__ void body_dir(const double* G, const double* x, double* d) {
  const double* a = G + 3;
  const double* Q = G + 6;
  double dx[3] = {x[0] - G[0], x[1] - G[1], x[2] - G[2]};
  for (int k = 0; k < 3; ++k) d[k] = (Q[k] * dx[0] + Q[3 + k] * dx[1] + Q[6 + k] * dx[2]) / a[k];
}

// partial normal equations of a least-squares SH fit, Y^T Y c = Y^T v: the
// lower triangle of Y^T Y (row-major, i >= j) followed by Y^T v, SH_E
// entries.  Workgroup (g, y) sums over the point tiles g, g + G, g + 2G, ...
// (G = gridDim.x) the entries y * FIT_EB ... of that list, four per thread.
// Points are either unit directions (dirs) or positions mapped to
// body-frame directions (pos + G).
constexpr int FIT_PTS = 64;
constexpr int FIT_EB = 1024;
constexpr int FIT_NB = 64;                       // at most this many point groups
constexpr int SH_T = SH_N * (SH_N + 1) / 2;
constexpr int SH_E = SH_T + SH_N;
constexpr int SH_EP = (SH_E + 255) / 256 * 256;  // partial stride (whole 256-entry rows)

// (i, j), i >= j, of entry e of the row-major lower triangle
__device__ __forceinline__ void tri_index(int e, int& i, int& j) {
  int r = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
  while (r * (r + 1) / 2 > e) --r;
  while ((r + 1) * (r + 2) / 2 <= e) ++r;
  i = r;
  j = e - r * (r + 1) / 2;
}

__global__ void __launch_bounds__(256) k_sh_normal(int n, const double* dirs, const double* pos, const double* G,
                                                   const double* vals, const float* valsf, double scale,
                                                   double* part) {
  __shared__ double Ys[FIT_PTS][SH_N + 1];       // column SH_N holds v
  int ei[4], ej[4];
  double s[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = blockIdx.y * FIT_EB + u * 256 + threadIdx.x;
    s[u] = 0.0;
    ei[u] = -1;
    ej[u] = 0;
    if (e < SH_T) {
      tri_index(e, ei[u], ej[u]);
    } else if (e < SH_E) {
      ei[u] = e - SH_T;
      ej[u] = SH_N;
    }
  }
  for (int p0 = blockIdx.x * FIT_PTS; p0 < n; p0 += gridDim.x * FIT_PTS) {
    const int np = n - p0 < FIT_PTS ? n - p0 : FIT_PTS;
    __syncthreads();
    for (int q = threadIdx.x; q < np; q += blockDim.x) {
      double d[3];
      if (dirs) {
        for (int k = 0; k < 3; ++k) d[k] = dirs[3 * (int64_t)(p0 + q) + k];
      } else {
        body_dir(G, pos + 3 * (int64_t)(p0 + q), d);
      }
      real_sh(d, Ys[q]);
      Ys[q][SH_N] = scale * (vals ? vals[p0 + q] : (double)valsf[p0 + q]);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (ei[u] >= 0)
        for (int q = 0; q < np; ++q) s[u] += Ys[q][ei[u]] * Ys[q][ej[u]];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = blockIdx.y * FIT_EB + u * 256 + threadIdx.x;
    if (e < SH_EP) part[(int64_t)blockIdx.x * SH_EP + e] = s[u];
  }
}

__device__ __forceinline__ double lane_bcast(double v, int l) {
  const long long u = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(u & 0xffffffffll), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// sum of the nb partial normal equations (fixed order), then the solve of
// the 81 x 81 symmetric positive definite system in one workgroup:
// right-looking LDL^T elimination (one barrier per pivot; each of 64 row
// slots x 4 column phases updates its share of the trailing lower
// triangle and the right-hand side), then back substitution with
// L^T D on wavefront 0 (rows in lanes, the solved unknown broadcast from
// its lane).  coef = (Y^T Y)^-1 Y^T v
__global__ void __launch_bounds__(256) k_sh_solve(int nb, const double* part, double* coef) {
  __shared__ double A[SH_N][SH_N + 1];
  __shared__ double b[SH_N];
  __shared__ double cb[2][SH_N];
  constexpr int EPT = SH_EP / 256;
  const int t = threadIdx.x;
  double s[EPT];
#pragma unroll
  for (int u = 0; u < EPT; ++u) s[u] = 0.0;
  // whole rows of the padded partials, two groups per pass so that their
  // loads are in flight together (the padding entries are zeros)
  int g = 0;
  for (; g + 1 < nb; g += 2) {
    const double* p0 = part + (int64_t)g * SH_EP + t;
    double v0[EPT], v1[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      v0[u] = p0[u * 256];
      v1[u] = p0[SH_EP + u * 256];
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u) s[u] += v0[u] + v1[u];
  }
  if (g < nb) {
    const double* p0 = part + (int64_t)g * SH_EP + t;
#pragma unroll
    for (int u = 0; u < EPT; ++u) s[u] += p0[u * 256];
  }
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int e = u * 256 + t;
    if (e < SH_T) {
      int i, j;
      tri_index(e, i, j);
      A[i][j] = s[u];
    } else if (e < SH_E) {
      b[e - SH_T] = s[u];
    }
  }
  // pivot column k is also kept in cb[k & 1] (a separate array, so its
  // reads do not wait on the trailing update's stores); after pivot k,
  // A[i][k] (i > k) holds L[i][k] d_k and b the forward-substituted
  // right-hand side; the diagonal holds d
  __syncthreads();
  if (t < SH_N) cb[0][t] = A[t][0];
  const int r = t >> 2, c = t & 3;
  for (int k = 0; k < SH_N; ++k) {
    __syncthreads();
    const double* ck = cb[k & 1];
    double* cn = cb[(k + 1) & 1];
    const double inv = 1.0 / ck[k];
    const double bk = b[k];
    for (int i = k + 1 + r; i < SH_N; i += 64) {
      const double f = ck[i] * inv;
      double* Ai = A[i];
      // columns j0, j0 + 4, ... <= i, eight at a time: the loads of a
      // chunk are unconditional (column clamped to i, in the row) and all
      // issued before its stores, which are the only guarded accesses
      const int j0 = k + 1 + c;
      const int nj = j0 <= i ? (i - j0) / 4 + 1 : 0;
      double first = 0.0;
      for (int m = 0; m < nj; m += 8) {
        double av[8], cv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int j = min(j0 + 4 * (m + u), i);
          av[u] = Ai[j];
          cv[u] = ck[j];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (m + u < nj) {
            const double v = av[u] - f * cv[u];
            Ai[j0 + 4 * (m + u)] = v;
            if (m + u == 0) first = v;
          }
      }
      if (c == 0) {
        cn[i] = first;
        b[i] -= f * bk;
      }
    }
  }
  __syncthreads();
  if (t >= 64) return;
  // x_i = (y_i - sum_{j > i} A[j][i] x_j) / d_i, lanes own rows t and t + 64
  const int i0 = t, i1 = t + 64;
  const bool h1 = i1 < SH_N;
  double a0 = b[i0], a1 = h1 ? b[i1] : 0.0;
  const double r0 = 1.0 / A[i0][i0], r1 = h1 ? 1.0 / A[i1][i1] : 0.0;
  for (int j = SH_N - 1; j > 0; --j) {
    const double xj = lane_bcast(j >= 64 ? a1 * r1 : a0 * r0, j & 63);
    if (i0 < j) a0 -= A[j][i0] * xj;
    if (h1 && i1 < j) a1 -= A[j][i1] * xj;
  }
  coef[i0] = a0 * r0;
  if (h1) coef[i1] = a1 * r1;
}

// values of the SH expansion at points (unit directions or body-frame
// directions of positions): out double and/or float (times oscale)
__global__ void k_sh_eval(int n, const double* dirs, const double* pos, const double* G, const double* coef,
                          double* out, float* outf, double oscale) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  double d[3];
  if (dirs) {
    for (int k = 0; k < 3; ++k) d[k] = dirs[3 * (int64_t)q + k];
  } else {
    body_dir(G, pos + 3 * (int64_t)q, d);
  }
  double Y[SH_N];
  real_sh(d, Y);
  double s = 0.0;
  for (int i = 0; i < SH_N; ++i) s += Y[i] * coef[i];
  if (out) out[q] = s * oscale;
  if (outf) outf[q] = (float)(s * oscale);
}

inline unsigned nbl(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// ======================================================================== MLP object
struct kfbi_mlp {
  hipStream_t stream;
  int L;                              // layers
  std::vector<int> w;                 // widths, L + 1
  int64_t n_params, n_wbf;
  std::vector<int64_t> off_w, off_b, off_wb;   // offsets in the fp32 pack / bf16 copy
  float *p, *m, *v, *g;               // fp32 master, Adam moments, gradient
  uint16_t* wb;                       // bf16 weight copies
  int64_t* bf_index;
  int64_t step;
  // activations for a batch of up to cap rows
  int cap;
  std::vector<uint16_t*> a_b;         // bf16 inputs of every layer (L)
  std::vector<float*> z;              // fp32 pre-activations (L)
  float *dz, *da;
  uint16_t* dzb;
  float *y, *dy;                      // linear head: output and its gradient
  double* part;
  float* gv;                          // slab partials of the few-row forward
  float* sk;                          // split-K partials of the weight gradients
  float* cs;                          // row-slab partials of the bias gradients
};

namespace {

template <typename T>
kfbi_status dalloc_t(T** p, int64_t n) {
  *p = nullptr;
  if (hipMalloc((void**)p, (size_t)(n < 1 ? 1 : n) * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    kfbi_set_error("device allocation of %lld bytes failed", (long long)(n * sizeof(T)));
    return KFBI_E_OOM;
  }
  return KFBI_OK;
}

template <typename T>
void dfree_t(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

void free_batch(kfbi_mlp* h) {
  for (auto& x : h->a_b) dfree_t(x);
  for (auto& x : h->z) dfree_t(x);
  dfree_t(h->dz);
  dfree_t(h->da);
  dfree_t(h->dzb);
  dfree_t(h->y);
  dfree_t(h->dy);
  dfree_t(h->part);
  dfree_t(h->gv);
  dfree_t(h->sk);
  dfree_t(h->cs);
  h->cap = 0;
}

kfbi_status ensure_batch(kfbi_mlp* h, int B) {
  if (B <= h->cap) return KFBI_OK;
  free_batch(h);
  int maxw = 0;
  for (int x : h->w) maxw = x > maxw ? x : maxw;
  for (int l = 0; l < h->L; ++l) {
    KCHK(dalloc_t(&h->a_b[l], (int64_t)B * h->w[l]));
    KCHK(dalloc_t(&h->z[l], (int64_t)B * h->w[l + 1]));
  }
  KCHK(dalloc_t(&h->dz, (int64_t)B * maxw));
  KCHK(dalloc_t(&h->da, (int64_t)B * maxw));
  KCHK(dalloc_t(&h->dzb, (int64_t)B * maxw));
  KCHK(dalloc_t(&h->y, (int64_t)B * maxw));
  KCHK(dalloc_t(&h->dy, (int64_t)B * maxw));
  KCHK(dalloc_t(&h->part, 1024));
  int64_t gv = 0;
  for (int l = 0; l < h->L; ++l) {
    const int64_t n = (int64_t)GV_BMAX * h->w[l + 1] * ((h->w[l] + GV_KC - 1) / GV_KC);
    gv = n > gv ? n : gv;
  }
  KCHK(dalloc_t(&h->gv, gv));
  int64_t mn = 0, wmax = 0;
  for (int l = 0; l < h->L; ++l) {
    mn = std::max(mn, (int64_t)h->w[l] * h->w[l + 1]);
    wmax = std::max(wmax, (int64_t)h->w[l + 1]);
  }
  KCHK(dalloc_t(&h->sk, (int64_t)SK_MAX * mn));
  KCHK(dalloc_t(&h->cs, (int64_t)CS_SLABS * wmax));
  h->cap = B;
  return KFBI_OK;
}

template <bool AT, bool BT>
void gemm(hipStream_t st, int M, int N, int K, const uint16_t* A, int lda, const uint16_t* B, int ldb,
          const float* bias, const float* z, int relu_b, float* Cf, uint16_t* Cb, int ldc) {
  GemmArgs g{M, N, K, lda, ldb, ldc, A, B, bias, z, relu_b, Cf, Cb,
             lda % 8 == 0 && ((uintptr_t)A & 15) == 0, ldb % 8 == 0 && ((uintptr_t)B & 15) == 0, K, 0};
  dim3 grid((unsigned)((N + GBN - 1) / GBN), (unsigned)((M + GBM - 1) / GBM));
  hipLaunchKernelGGL((k_gemm<AT, BT>), grid, dim3(256), 0, st, g);
}

// C [M x N] (row stride N, no epilogue) with K split over up to SK_MAX work
// groups per tile when the tiles alone leave most of the chip idle: each
// writes its partial product into ws, k_splitk_sum adds them in order
// (the weight gradients: M, N <= a few hundred, K = the batch rows)
template <bool AT, bool BT>
void gemm_splitk(hipStream_t st, int M, int N, int K, const uint16_t* A, int lda, const uint16_t* B, int ldb,
                 float* C, float* ws) {
  const int tiles = ((N + GBN - 1) / GBN) * ((M + GBM - 1) / GBM);
  int S = K >= 4 * GBK * 2 && tiles < 256 ? (256 + tiles - 1) / tiles : 1;
  if (S > SK_MAX) S = SK_MAX;
  if (S > K / (2 * GBK)) S = K / (2 * GBK);
  if (S <= 1) {
    gemm<AT, BT>(st, M, N, K, A, lda, B, ldb, nullptr, nullptr, 0, C, nullptr, N);
    return;
  }
  const int kchunk = ((K + S - 1) / S + GBK - 1) / GBK * GBK;
  S = (K + kchunk - 1) / kchunk;
  GemmArgs g{M, N, K, lda, ldb, N, A, B, nullptr, nullptr, 0, ws, nullptr,
             lda % 8 == 0 && ((uintptr_t)A & 15) == 0, ldb % 8 == 0 && ((uintptr_t)B & 15) == 0, kchunk,
             (int64_t)M * N};
  dim3 grid((unsigned)((N + GBN - 1) / GBN), (unsigned)((M + GBM - 1) / GBM), (unsigned)S);
  hipLaunchKernelGGL((k_gemm<AT, BT>), grid, dim3(256), 0, st, g);
  const int64_t n = (int64_t)M * N;
  hipLaunchKernelGGL(k_splitk_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, S, n, (const float*)ws,
                     C);
}

// forward pass of B rows; X fp32 [B x w0]; the output is z[L-1]
void forward(kfbi_mlp* h, const float* X, int B) {
  hipStream_t st = h->stream;
  hipLaunchKernelGGL(k_to_bf16, dim3(nbl((int64_t)B * h->w[0])), dim3(256), 0, st, (int64_t)B * h->w[0], X,
                     h->a_b[0]);
  for (int l = 0; l < h->L; ++l) {
    const bool last = l == h->L - 1;
    // z_l = a_l W_l + b_l (fp32, kept for the backward mask) and
    // a_{l+1} = relu(z_l) (bf16, the next layer's operand)
    const int K = h->w[l], N = h->w[l + 1];
    if (B <= GV_BMAX && N % 8 == 0 && h->off_wb[l] % 8 == 0) {
      const int nch = (K + GV_KC - 1) / GV_KC;
      hipLaunchKernelGGL(k_gemv_part, dim3((unsigned)((N + GV_COLS - 1) / GV_COLS), (unsigned)nch), dim3(256), 0, st,
                         B, N, K, (const uint16_t*)h->a_b[l], K, (const uint16_t*)(h->wb + h->off_wb[l]), N, h->gv);
      hipLaunchKernelGGL(k_gemv_sum, dim3(nbl((int64_t)B * N, 4)), dim3(256), 0, st, B * N, N, nch,
                         (const float*)h->gv, (const float*)(h->p + h->off_b[l]), 1, h->z[l],
                         last ? nullptr : h->a_b[l + 1]);
    } else {
      gemm<false, false>(st, B, N, K, h->a_b[l], K, h->wb + h->off_wb[l], N, h->p + h->off_b[l], nullptr, 1, h->z[l],
                         last ? nullptr : h->a_b[l + 1], N);
    }
  }
}

// gradient into h->g from the output gradient in h->dz / h->dzb
void backward_from(kfbi_mlp* h, int B) {
  hipStream_t st = h->stream;
  const int L = h->L;
  for (int l = L - 1; l >= 0; --l) {
    const int in = h->w[l], out = h->w[l + 1];
    // dW_l = a_l^T dz (fp32 into the gradient pack), db_l = column sums of dz
    gemm_splitk<true, false>(st, in, out, B, h->a_b[l], in, h->dzb, out, h->g + h->off_w[l], h->sk);
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)((out + 63) / 64), CS_SLABS), dim3(256), 0, st, B, out,
                       (const float*)h->dz, h->cs);
    hipLaunchKernelGGL(k_colsum_final, dim3(nbl(out)), dim3(256), 0, st, out, CS_SLABS, (const float*)h->cs,
                       h->g + h->off_b[l]);
    if (l > 0) {
      // dz_{l-1} = (dz W_l^T) masked by z_{l-1} > 0
      gemm<false, true>(st, B, in, out, h->dzb, out, h->wb + h->off_wb[l], out, nullptr, h->z[l - 1], 0, h->da,
                        nullptr, in);
      std::swap(h->dz, h->da);
      hipLaunchKernelGGL(k_to_bf16, dim3(nbl((int64_t)B * in)), dim3(256), 0, st, (int64_t)B * in,
                         (const float*)h->dz, h->dzb);
    }
  }
}

// loss and gradient into h->g; loss (device float)
void backward(kfbi_mlp* h, const float* Yt, int B, float* loss) {
  hipStream_t st = h->stream;
  const int L = h->L;
  const int64_t no = (int64_t)B * h->w[L];
  unsigned nbk = nbl(no);
  if (nbk > 1024) nbk = 1024;
  hipLaunchKernelGGL(k_mse, dim3(nbk), dim3(256), 0, st, no, h->z[L - 1], Yt, h->dz, h->dzb, h->part);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, st, (int)nbk, no, (const double*)h->part, loss);
  backward_from(h, B);
}

// linear head: loss of y = head(z, C) against Yt and the gradient into h->g
// (h->y and h->dy hold the head's output and output gradient)
// B examples of R rows each: the output of example b is its R rows read as
// one row of R w_L entries
void backward_lin(kfbi_mlp* h, const float* C, int nb, const float* Yt, int B, int R, float* loss) {
  hipStream_t st = h->stream;
  const int L = h->L;
  const int K = R * h->w[L] / nb;
  const int64_t ny = (int64_t)B * K;
  hipLaunchKernelGGL(k_lin_head_fwd, dim3(nbl(ny)), dim3(256), 0, st, B, nb, K, C, (const float*)h->z[L - 1], h->y);
  unsigned nbk = nbl(ny);
  if (nbk > 1024) nbk = 1024;
  // dy = 2 (y - Yt) / n (bf16 copy into dzb, unused) and the loss
  hipLaunchKernelGGL(k_mse, dim3(nbk), dim3(256), 0, st, ny, (const float*)h->y, Yt, h->dy, h->dzb, h->part);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, st, (int)nbk, ny, (const double*)h->part, loss);
  hipLaunchKernelGGL(k_lin_head_bwd, dim3(nbl((int64_t)B * R * h->w[L])), dim3(256), 0, st, B, nb, K, C,
                     (const float*)h->dy, h->dz, h->dzb);
  backward_from(h, B * R);
}

void adam_step(kfbi_mlp* h, float lr) {
  h->step += 1;
  AdamArgs a;
  a.n = h->n_params;
  a.lr = lr;
  a.b1 = 0.9f;
  a.b2 = 0.999f;
  a.eps = 1e-8f;
  a.c1 = (float)(1.0 - pow(0.9, (double)h->step));
  a.c2 = (float)(1.0 - pow(0.999, (double)h->step));
  a.w = h->p;
  a.m = h->m;
  a.v = h->v;
  a.g = h->g;
  a.bf_index = h->bf_index;
  a.wb = h->wb;
  hipLaunchKernelGGL(k_adam, dim3(nbl(h->n_params)), dim3(256), 0, h->stream, a);
}

}  // namespace

extern "C" kfbi_status kfbi_mlp_create(int n_layers, const int* widths, void* stream, kfbi_mlp** out) {
  if (!out || !widths || n_layers < 1 || n_layers > 16) {
    kfbi_set_error("mlp needs 1..16 layers and a width list");
    return KFBI_E_INVALID;
  }
  for (int i = 0; i <= n_layers; ++i)
    if (widths[i] < 1 || widths[i] > (1 << 20)) {
      kfbi_set_error("mlp width %d out of range", widths[i]);
      return KFBI_E_INVALID;
    }
  kfbi_mlp* h = new (std::nothrow) kfbi_mlp();
  if (!h) return KFBI_E_OOM;
  h->stream = (hipStream_t)stream;
  h->L = n_layers;
  h->w.assign(widths, widths + n_layers + 1);
  int64_t np = 0, nb = 0;
  for (int l = 0; l < n_layers; ++l) {
    h->off_w.push_back(np);
    np += (int64_t)widths[l] * widths[l + 1];
    h->off_b.push_back(np);
    np += widths[l + 1];
    h->off_wb.push_back(nb);
    nb += (int64_t)widths[l] * widths[l + 1];
  }
  h->n_params = np;
  h->n_wbf = nb;
  h->a_b.assign(n_layers, nullptr);
  h->z.assign(n_layers, nullptr);
  kfbi_status st = KFBI_OK;
  if ((st = dalloc_t(&h->p, np)) || (st = dalloc_t(&h->m, np)) || (st = dalloc_t(&h->v, np)) ||
      (st = dalloc_t(&h->g, np)) || (st = dalloc_t(&h->wb, nb)) || (st = dalloc_t(&h->bf_index, np))) {
    kfbi_mlp_destroy(h);
    return st;
  }
  std::vector<int64_t> idx((size_t)np, -1);
  for (int l = 0; l < n_layers; ++l)
    for (int64_t i = 0; i < (int64_t)widths[l] * widths[l + 1]; ++i) idx[(size_t)(h->off_w[l] + i)] = h->off_wb[l] + i;
  if (hipMemcpy(h->bf_index, idx.data(), sizeof(int64_t) * np, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(h->p, 0, sizeof(float) * np) != hipSuccess || hipMemset(h->m, 0, sizeof(float) * np) != hipSuccess ||
      hipMemset(h->v, 0, sizeof(float) * np) != hipSuccess || hipMemset(h->wb, 0, 2 * nb) != hipSuccess) {
    (void)hipGetLastError();
    kfbi_set_error("mlp initialisation copy failed");
    kfbi_mlp_destroy(h);
    return KFBI_E_DEVICE;
  }
  *out = h;
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_mlp_sizes(const kfbi_mlp* h, int64_t* n_params) {
  if (!h || !n_params) {
    kfbi_set_error("mlp is NULL");
    return KFBI_E_INVALID;
  }
  *n_params = h->n_params;
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_mlp_set_params(kfbi_mlp* h, const float* params) {
  if (!h || !params) {
    kfbi_set_error("mlp or params is NULL");
    return KFBI_E_INVALID;
  }
  HIPCHK(hipMemcpyAsync(h->p, params, sizeof(float) * h->n_params, hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(hipMemsetAsync(h->m, 0, sizeof(float) * h->n_params, h->stream));
  HIPCHK(hipMemsetAsync(h->v, 0, sizeof(float) * h->n_params, h->stream));
  hipLaunchKernelGGL(k_refresh_bf16, dim3(nbl(h->n_params)), dim3(256), 0, h->stream, h->n_params,
                     (const float*)h->p, (const int64_t*)h->bf_index, h->wb);
  h->step = 0;
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_mlp_get_params(const kfbi_mlp* h, float* params) {
  if (!h || !params) {
    kfbi_set_error("mlp or params is NULL");
    return KFBI_E_INVALID;
  }
  HIPCHK(hipMemcpyAsync(params, h->p, sizeof(float) * h->n_params, hipMemcpyDeviceToDevice, h->stream));
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_mlp_forward(kfbi_mlp* h, const float* X, int B, float* Y) {
  if (!h || !X || !Y || B < 1) {
    kfbi_set_error("mlp forward needs X, Y and B >= 1");
    return KFBI_E_INVALID;
  }
  KCHK(ensure_batch(h, B));
  forward(h, X, B);
  HIPCHK(hipMemcpyAsync(Y, h->z[h->L - 1], sizeof(float) * (size_t)B * h->w[h->L], hipMemcpyDeviceToDevice,
                        h->stream));
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_mlp_loss_grad(kfbi_mlp* h, const float* X, const float* Yt, int B, float* loss,
                                          float* grads) {
  if (!h || !X || !Yt || !loss || B < 1) {
    kfbi_set_error("mlp loss_grad needs X, Yt, loss and B >= 1");
    return KFBI_E_INVALID;
  }
  KCHK(ensure_batch(h, B));
  forward(h, X, B);
  backward(h, Yt, B, loss);
  if (grads)
    HIPCHK(hipMemcpyAsync(grads, h->g, sizeof(float) * h->n_params, hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_mlp_train_step(kfbi_mlp* h, const float* X, const float* Yt, int B, float lr,
                                           float* loss) {
  if (!h || !X || !Yt || !loss || B < 1 || !(lr > 0.f)) {
    kfbi_set_error("mlp train_step needs X, Yt, loss, B >= 1 and lr > 0");
    return KFBI_E_INVALID;
  }
  KCHK(ensure_batch(h, B));
  forward(h, X, B);
  backward(h, Yt, B, loss);
  adam_step(h, lr);
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

namespace {
kfbi_status lin_check(const kfbi_mlp* h, const float* X, const float* C, int nb, int B, int R) {
  if (!h || !X || !C || B < 1 || R < 1 || nb < 1 || ((int64_t)R * h->w[h->L]) % nb != 0) {
    kfbi_set_error("linear head needs X, C, B >= 1, R >= 1 and nb dividing R times the output width");
    return KFBI_E_INVALID;
  }
  return KFBI_OK;
}
}  // namespace

extern "C" kfbi_status kfbi_mlp_forward_lin(kfbi_mlp* h, const float* X, int B, int R, const float* C, int nb,
                                            float* Y) {
  KCHK(lin_check(h, X, C, nb, B, R));
  if (!Y) {
    kfbi_set_error("forward_lin needs an output");
    return KFBI_E_INVALID;
  }
  KCHK(ensure_batch(h, B * R));
  forward(h, X, B * R);
  const int K = R * h->w[h->L] / nb;
  hipLaunchKernelGGL(k_lin_head_fwd, dim3(nbl((int64_t)B * K)), dim3(256), 0, h->stream, B, nb, K, C,
                     (const float*)h->z[h->L - 1], Y);
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_mlp_loss_grad_lin(kfbi_mlp* h, const float* X, int B, int R, const float* C, int nb,
                                              const float* Yt, float* loss, float* grads) {
  KCHK(lin_check(h, X, C, nb, B, R));
  if (!Yt || !loss) {
    kfbi_set_error("loss_grad_lin needs targets and a loss");
    return KFBI_E_INVALID;
  }
  KCHK(ensure_batch(h, B * R));
  forward(h, X, B * R);
  backward_lin(h, C, nb, Yt, B, R, loss);
  if (grads)
    HIPCHK(hipMemcpyAsync(grads, h->g, sizeof(float) * h->n_params, hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_mlp_train_step_lin(kfbi_mlp* h, const float* X, int B, int R, const float* C, int nb,
                                               const float* Yt, float lr, float* loss) {
  KCHK(lin_check(h, X, C, nb, B, R));
  if (!Yt || !loss || !(lr > 0.f)) {
    kfbi_set_error("train_step_lin needs targets, a loss and lr > 0");
    return KFBI_E_INVALID;
  }
  KCHK(ensure_batch(h, B * R));
  forward(h, X, B * R);
  backward_lin(h, C, nb, Yt, B, R, loss);
  adam_step(h, lr);
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_geometry_input(const double* geom, int P, void* stream, float* X) {
  if (!geom || !X || P < 1) {
    kfbi_set_error("geometry_input needs geometries and outputs");
    return KFBI_E_INVALID;
  }
  hipLaunchKernelGGL(k_geom_input, dim3(nbl((int64_t)P * 8)), dim3(256), 0, (hipStream_t)stream, P, geom, X);
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_mlp_destroy(kfbi_mlp* h) {
  if (!h) return KFBI_OK;
  free_batch(h);
  dfree_t(h->p);
  dfree_t(h->m);
  dfree_t(h->v);
  dfree_t(h->g);
  dfree_t(h->wb);
  dfree_t(h->bf_index);
  delete h;
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_gemm_bf16(int transA, int transB, int M, int N, int K, const uint16_t* A, int lda,
                                      const uint16_t* B, int ldb, float* C, int ldc, void* stream) {
  if (M < 1 || N < 1 || K < 1 || !A || !B || !C) {
    kfbi_set_error("gemm needs positive sizes and buffers");
    return KFBI_E_INVALID;
  }
  hipStream_t st = (hipStream_t)stream;
  if (!transA && !transB)
    gemm<false, false>(st, M, N, K, A, lda, B, ldb, nullptr, nullptr, 0, C, nullptr, ldc);
  else if (transA && !transB)
    gemm<true, false>(st, M, N, K, A, lda, B, ldb, nullptr, nullptr, 0, C, nullptr, ldc);
  else if (!transA && transB)
    gemm<false, true>(st, M, N, K, A, lda, B, ldb, nullptr, nullptr, 0, C, nullptr, ldc);
  else {
    kfbi_set_error("gemm: both operands transposed is not supported");
    return KFBI_E_INVALID;
  }
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

// ======================================================================== features and transfer
extern "C" kfbi_status kfbi_scale_jumps(float* X, float* Y, const float* alpha, int B, int ns, int nout,
                                        void* stream) {
  if (!X || !Y || !alpha || B < 1 || ns < 1 || nout < 1) {
    kfbi_set_error("scale_jumps needs features, targets, factors and sizes");
    return KFBI_E_INVALID;
  }
  const int64_t n = (int64_t)B * ns * 2 + (int64_t)B * nout;
  hipLaunchKernelGGL(k_scale_jumps, dim3(nbl(n)), dim3(256), 0, (hipStream_t)stream, B, ns, nout, alpha, X, Y);
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_ellipsoid_features(const double* geom, const double* jumps, int P, const double* S,
                                               int ns, void* stream, float* X) {
  if (!geom || !jumps || !S || !X || P < 1 || ns < 1) {
    kfbi_set_error("features need geometry, jumps, samples and outputs");
    return KFBI_E_INVALID;
  }
  hipLaunchKernelGGL(k_features, dim3(nbl((int64_t)P * ns)), dim3(256), 0, (hipStream_t)stream, P, ns, geom, jumps,
                     S, X);
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

namespace {
// part [groups][SH_EP] and coef [SH_N] in ws (at least sh_ws_len(n_in) values)
int sh_groups(int n_in) {
  const int g = (n_in + FIT_PTS - 1) / FIT_PTS;
  return g < FIT_NB ? g : FIT_NB;
}

int64_t sh_ws_len(int n_in) { return (int64_t)sh_groups(n_in) * SH_EP + SH_N; }

void sh_fit_eval(hipStream_t st, double* ws, int n_in, const double* dirs_in, const double* pos_in,
                 const double* G, const double* vals, const float* valsf, double vscale, int n_out,
                 const double* dirs_out, const double* pos_out, double* out, float* outf, double oscale) {
  const int ng = sh_groups(n_in);
  double* part = ws;
  double* coef = ws + (int64_t)ng * SH_EP;
  hipLaunchKernelGGL(k_sh_normal, dim3(ng, (SH_E + FIT_EB - 1) / FIT_EB), dim3(256), 0, st, n_in, dirs_in, pos_in, G,
                     vals, valsf, vscale, part);
  hipLaunchKernelGGL(k_sh_solve, dim3(1), dim3(256), 0, st, ng, (const double*)part, coef);
  hipLaunchKernelGGL(k_sh_eval, dim3(nbl(n_out)), dim3(256), 0, st, n_out, dirs_out, pos_out, G,
                     (const double*)coef, out, outf, oscale);
}

// the plan's transfer workspace (grown, never shrunk; freed with the plan)
kfbi_status sh_workspace(kfbi_plan* pl, int64_t need, double** ws) {
  if (need > pl->sh_ws_cap) {
    if (pl->sh_ws) (void)hipFree(pl->sh_ws);
    pl->sh_ws = nullptr;
    pl->sh_ws_cap = 0;
    KCHK(dalloc_t(&pl->sh_ws, need));
    pl->sh_ws_cap = need;
  }
  *ws = pl->sh_ws;
  return KFBI_OK;
}
}  // namespace

extern "C" kfbi_status kfbi_sh_transfer(kfbi_plan* pl, const double* geom, const double* S, int ns,
                                        const float* psi_s, double scale, double* psi_dof) {
  if (!pl || !pl->ready || !geom || !S || !psi_s || !psi_dof || ns < (SH_N)) {
    kfbi_set_error("transfer needs a ready plan, geometry, >= 81 samples and outputs");
    return KFBI_E_INVALID;
  }
  if (pl->g.d != 3) {
    kfbi_set_error("the spherical-harmonic transfer is defined in 3D");
    return KFBI_E_INVALID;
  }
  // workspace: DOF positions (the surface table gathered through d2s), then
  // the fit's partial normal equations and coefficients; everything stays
  // ordered on the plan's stream
  double* ws = nullptr;
  KCHK(sh_workspace(pl, 3 * pl->n_dof + sh_ws_len(ns), &ws));
  double* dpos = ws;
  KCHK(kfbi_plan_export(pl, KFBI_EXPORT_DOF_POS, dpos, (int64_t)sizeof(double) * 3 * pl->n_dof));
  sh_fit_eval(pl->stream, ws + 3 * pl->n_dof, ns, S, nullptr, geom, nullptr, psi_s, scale, (int)pl->n_dof, nullptr,
              dpos, psi_dof, nullptr, 1.0);
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_sh_sample(kfbi_plan* pl, const double* geom, const double* psi_dof, const double* S,
                                      int ns, double scale, float* psi_s) {
  if (!pl || !pl->ready || !geom || !S || !psi_s || !psi_dof || ns < 1 || pl->n_dof < SH_N) {
    kfbi_set_error("sampling needs a ready plan with >= 81 DOFs, geometry, samples and outputs");
    return KFBI_E_INVALID;
  }
  if (pl->g.d != 3) {
    kfbi_set_error("the spherical-harmonic transfer is defined in 3D");
    return KFBI_E_INVALID;
  }
  double* ws = nullptr;
  KCHK(sh_workspace(pl, 3 * pl->n_dof + sh_ws_len((int)pl->n_dof), &ws));
  double* dpos = ws;
  KCHK(kfbi_plan_export(pl, KFBI_EXPORT_DOF_POS, dpos, (int64_t)sizeof(double) * 3 * pl->n_dof));
  sh_fit_eval(pl->stream, ws + 3 * pl->n_dof, (int)pl->n_dof, nullptr, dpos, geom, psi_dof, nullptr, 1.0, ns, S,
              nullptr, nullptr, psi_s, scale);
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_sh_coefficients(kfbi_plan* pl, const double* geom, const double* psi_dof, double scale,
                                            double* coef) {
  if (!pl || !pl->ready || !geom || !psi_dof || !coef || pl->n_dof < SH_N) {
    kfbi_set_error("SH coefficients need a ready plan with >= 81 DOFs, geometry, density and output");
    return KFBI_E_INVALID;
  }
  if (pl->g.d != 3) {
    kfbi_set_error("the spherical-harmonic transfer is defined in 3D");
    return KFBI_E_INVALID;
  }
  double* ws = nullptr;
  const int n = (int)pl->n_dof;
  KCHK(sh_workspace(pl, 3 * pl->n_dof + sh_ws_len(n), &ws));
  double* dpos = ws;
  KCHK(kfbi_plan_export(pl, KFBI_EXPORT_DOF_POS, dpos, (int64_t)sizeof(double) * 3 * pl->n_dof));
  double* fw = ws + 3 * pl->n_dof;
  const int ng = sh_groups(n);
  hipLaunchKernelGGL(k_sh_normal, dim3(ng, (SH_E + FIT_EB - 1) / FIT_EB), dim3(256), 0, pl->stream, n,
                     (const double*)nullptr, (const double*)dpos, geom, psi_dof, (const float*)nullptr, scale, fw);
  hipLaunchKernelGGL(k_sh_solve, dim3(1), dim3(256), 0, pl->stream, ng, (const double*)fw, coef);
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_sh_expand(kfbi_plan* pl, const double* geom, const double* coef, double scale,
                                      double* psi_dof) {
  if (!pl || !pl->ready || !geom || !coef || !psi_dof) {
    kfbi_set_error("SH expansion needs a ready plan, geometry, coefficients and output");
    return KFBI_E_INVALID;
  }
  if (pl->g.d != 3) {
    kfbi_set_error("the spherical-harmonic transfer is defined in 3D");
    return KFBI_E_INVALID;
  }
  double* ws = nullptr;
  KCHK(sh_workspace(pl, 3 * pl->n_dof, &ws));
  KCHK(kfbi_plan_export(pl, KFBI_EXPORT_DOF_POS, ws, (int64_t)sizeof(double) * 3 * pl->n_dof));
  hipLaunchKernelGGL(k_sh_eval, dim3(nbl(pl->n_dof)), dim3(256), 0, pl->stream, (int)pl->n_dof,
                     (const double*)nullptr, (const double*)ws, geom, coef, psi_dof, (float*)nullptr, scale);
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_learned_start(kfbi_plan* pl, kfbi_mlp* h, int nb, const double* geom,
                                          const double* jumps, double scale, double* psi_dof) {
  if (!pl || !pl->ready || !h || !geom || !jumps || !psi_dof || nb != 32 || h->w[0] != GEOM_IN ||
      h->w[h->L] != 4 * SH_N) {
    kfbi_set_error("learned start needs a ready plan, a network 15 -> ... -> 4 x 81, nb = 32 jump coefficients, "
                   "geometry and output");
    return KFBI_E_INVALID;
  }
  if (pl->g.d != 3) {
    kfbi_set_error("the learned start is defined in 3D");
    return KFBI_E_INVALID;
  }
  // workspace: DOF positions, the 81 coefficients, the network input
  double* ws = nullptr;
  KCHK(sh_workspace(pl, 3 * pl->n_dof + SH_N + 4 * GEOM_IN, &ws));
  double* dpos = ws;
  double* coef = ws + 3 * pl->n_dof;
  float* X = reinterpret_cast<float*>(coef + SH_N);
  KCHK(kfbi_plan_export(pl, KFBI_EXPORT_DOF_POS, dpos, (int64_t)sizeof(double) * 3 * pl->n_dof));
  KCHK(ensure_batch(h, 8));
  hipStream_t keep = h->stream;
  h->stream = pl->stream;     // the network's kernels go on the plan's stream
  hipLaunchKernelGGL(k_geom_input, dim3(1), dim3(64), 0, pl->stream, 1, geom, X);
  forward(h, X, 8);           // one row per Fourier mode
  hipLaunchKernelGGL(k_lin_head_coef, dim3(1), dim3(128), 0, pl->stream, SH_N, jumps, (const float*)h->z[h->L - 1],
                     scale, coef);
  hipLaunchKernelGGL(k_sh_eval, dim3(nbl(pl->n_dof)), dim3(256), 0, pl->stream, (int)pl->n_dof,
                     (const double*)nullptr, (const double*)dpos, geom, (const double*)coef, psi_dof, (float*)nullptr,
                     1.0);
  h->stream = keep;
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_real_sh(const double* dirs, int n, void* stream, double* Y) {
  if (!dirs || !Y || n < 1) {
    kfbi_set_error("real_sh needs directions and output");
    return KFBI_E_INVALID;
  }
  // evaluate each basis function as an expansion with a unit coefficient
  double* coef = nullptr;
  KCHK(dalloc_t(&coef, SH_N));
  hipStream_t st = (hipStream_t)stream;
  std::vector<double> e(SH_N, 0.0);
  kfbi_status rs = KFBI_OK;
  for (int i = 0; i < SH_N && rs == KFBI_OK; ++i) {
    e.assign(SH_N, 0.0);
    e[i] = 1.0;
    if (hipMemcpyAsync(coef, e.data(), sizeof(double) * SH_N, hipMemcpyHostToDevice, st) != hipSuccess) {
      rs = KFBI_E_DEVICE;
      break;
    }
    hipLaunchKernelGGL(k_sh_eval, dim3(nbl(n)), dim3(256), 0, st, n, dirs, (const double*)nullptr,
                       (const double*)nullptr, (const double*)coef, Y + (int64_t)i * n, (float*)nullptr, 1.0);
    if (hipStreamSynchronize(st) != hipSuccess) rs = KFBI_E_DEVICE;
  }
  dfree_t(coef);
  if (rs != KFBI_OK) kfbi_set_error("real_sh failed");
  return rs;
}
