// Small dense FP64 linear algebra on the device: one-sided Jacobi SVD,
// Cholesky with inverse, and element-wise helpers.  One workgroup works on
// one (small) matrix; batches run as a grid of workgroups.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// ---------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi SVD.  Columns of the m x n work matrix (column
// major, contiguous columns) are orthogonalised by plane rotations in
// round-robin order: n-1 rounds of n/2 disjoint column pairs per sweep, one
// wave per pair.  The rotation for columns p, q with a = |x_p|^2,
// b = |x_q|^2, g = x_p . x_q is t = sign(z) / (|z| + sqrt(1 + z^2)),
// z = (b - a) / (2 g), c = 1/sqrt(1 + t^2), s = c t; it makes the pair
// orthogonal.  Sweeps stop when every |g| <= tol sqrt(a b).
// ---------------------------------------------------------------------------
constexpr int SVD_THREADS = 1024;
constexpr int SVD_WAVES = SVD_THREADS / 64;

// GLOBAL_WORK false: the m x n work matrix and the n x n rotation accumulator
// live in dynamic LDS; otherwise in the global buffer `work`.  The choice is
// a template parameter so that the LDS pointers are known to be LDS and the
// accesses compile to LDS instructions rather than generic (flat) ones.
// Singular values (column norms of the converged X), sorted descending with
// ties by index, left vectors normalised and sign-fixed (the first entry
// within a relative 1e-8 of the largest magnitude is made positive), right
// vectors from the accumulated rotations W.
__device__ __forceinline__ void jacobi_emit(const double* X, int ldx, const double* W, int ldw, int m, int n,
                            double* colnorm, int* perm, long long b, double* __restrict__ U,
                            int ldu, long long sU, double* __restrict__ S, long long sS,
                            double* __restrict__ V, int ldv, long long sV) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nwave = (int)blockDim.x >> 6;
  // column norms = singular values
  for (int j = wave; j < n; j += nwave) {
    double a = 0.0;
    for (int i = lane; i < m; i += 64) a += X[(long long)j * ldx + i] * X[(long long)j * ldx + i];
    a = wave_sum(a);
    if (lane == 0) colnorm[j] = sqrt(a);
  }
  __syncthreads();
  // rank sort, descending, ties by index
  for (int j = tid; j < n; j += (int)blockDim.x) {
    int rank = 0;
    const double sj = colnorm[j];
    for (int i = 0; i < n; ++i) {
      const double si = colnorm[i];
      rank += (si > sj) || (si == sj && i < j);
    }
    perm[rank] = j;
  }
  __syncthreads();
  // outputs; each left vector sign-fixed (largest-magnitude entry positive)
  for (int r = wave; r < n; r += nwave) {
    const int j = perm[r];
    const double sj = colnorm[j];
    const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
    // sign: the first entry within a relative 1e-8 of the largest magnitude
    double best = 0.0;
    for (int i = lane; i < m; i += 64) best = fmax(best, fabs(X[(long long)j * ldx + i]));
    best = wave_max(best);
    int bi = 0x7fffffff;
    for (int i = lane; i < m; i += 64)
      if (fabs(X[(long long)j * ldx + i]) >= (1.0 - 1e-8) * best) {
        bi = i;
        break;
      }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) bi = min(bi, __shfl_xor(bi, o, 64));
    const double sg = (bi < m && X[(long long)j * ldx + bi] < 0.0) ? -1.0 : 1.0;
    if (U)
      for (int i = lane; i < m; i += 64)
        U[b * sU + (long long)i * ldu + r] = sg * inv * X[(long long)j * ldx + i];
    if (V)
      for (int i = lane; i < n; i += 64)
        V[b * sV + (long long)i * ldv + r] = sg * W[(long long)j * ldw + i];
    if (S && lane == 0) S[b * sS + r] = sj;
  }
}

template <bool GLOBAL_WORK>
__global__ __launch_bounds__(SVD_THREADS) void jacobi_svd_kernel(
    const double* __restrict__ Ain, int lda, long long sA, double* __restrict__ U, int ldu,
    long long sU, double* __restrict__ S, long long sS, double* __restrict__ V, int ldv,
    long long sV, int m, int n, double* __restrict__ work, int max_sweeps, double tol,
    unsigned long long* __restrict__ sweep_count) {
  extern __shared__ double lds[];
  const long long b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double* A = Ain + b * sA;
  // columns padded to an odd number of doubles so that the columns the
  // groups of one wave touch fall on different LDS banks
  const int ldx = m | 1, ldw = n | 1;
  double* X;  // X[j*ldx + i]
  if constexpr (GLOBAL_WORK)
    X = work + b * (long long)(ldx * n + ldw * n);
  else
    X = lds;
  double* W = X + (long long)ldx * n;  // W[j*ldw + i] (V columns)
  __shared__ double colnorm[512];
  __shared__ int perm[512];
  __shared__ int done;

  for (long long t = tid; t < (long long)m * n; t += SVD_THREADS) {
    const int i = (int)(t / n), j = (int)(t % n);
    X[(long long)j * ldx + i] = A[(long long)i * lda + j];
  }
  for (long long t = tid; t < (long long)n * n; t += SVD_THREADS) {
    const int i = (int)(t / n), j = (int)(t % n);
    W[(long long)j * ldw + i] = (i == j) ? 1.0 : 0.0;
  }
  if (tid == 0) done = 0;
  __syncthreads();

  // 16-lane groups: one column pair per group per round (64 groups); a lane
  // keeps its entries of the pair in registers between the dot products and
  // the rotation when m <= 16 * JREG
  constexpr int JREG = 8;
  const int grp = tid >> 4, gl = tid & 15;
  constexpr int NGRP = SVD_THREADS / 16;
  __shared__ double off_g[NGRP];
  const int N = (n + 1) & ~1;  // players incl. a dummy when n is odd
  const bool regs = m <= 16 * JREG;
  for (int sweep = 0; sweep < max_sweeps && n > 1; ++sweep) {
    double offmax = 0.0;
    for (int r = 0; r < N - 1; ++r) {
      for (int q = grp; q < N / 2; q += NGRP) {
        const int p0 = (q == 0) ? 0 : 1 + ((q - 1 + r) % (N - 1));
        const int p1 = 1 + ((N - 2 - q + r) % (N - 1));
        if (p0 >= n || p1 >= n) continue;
        const int p = min(p0, p1), qq = max(p0, p1);
        double* xp = X + (long long)p * ldx;
        double* xq = X + (long long)qq * ldx;
        double a = 0.0, bb = 0.0, g = 0.0;
        double up[JREG], vq[JREG];
        if (regs) {
#pragma unroll
          for (int e = 0; e < JREG; ++e) {
            const int i = gl + 16 * e;
            up[e] = i < m ? xp[i] : 0.0;
            vq[e] = i < m ? xq[i] : 0.0;
          }
#pragma unroll
          for (int e = 0; e < JREG; ++e) {
            a += up[e] * up[e];
            bb += vq[e] * vq[e];
            g += up[e] * vq[e];
          }
        } else {
          for (int i = gl; i < m; i += 16) {
            const double u = xp[i], v = xq[i];
            a += u * u;
            bb += v * v;
            g += u * v;
          }
        }
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) {
          a += __shfl_xor(a, o, 16);
          bb += __shfl_xor(bb, o, 16);
          g += __shfl_xor(g, o, 16);
        }
        const double scale = sqrt(a * bb);
        if (scale == 0.0 || fabs(g) <= tol * scale) continue;
        offmax = fmax(offmax, fabs(g) / scale);
        const double z = (bb - a) / (2.0 * g);
        const double t = (z >= 0.0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        if (regs) {
#pragma unroll
          for (int e = 0; e < JREG; ++e) {
            const int i = gl + 16 * e;
            if (i < m) {
              xp[i] = c * up[e] - s * vq[e];
              xq[i] = s * up[e] + c * vq[e];
            }
          }
        } else {
          for (int i = gl; i < m; i += 16) {
            const double u = xp[i], v = xq[i];
            xp[i] = c * u - s * v;
            xq[i] = s * u + c * v;
          }
        }
        double* wp = W + (long long)p * ldw;
        double* wq = W + (long long)qq * ldw;
        for (int i = gl; i < n; i += 16) {
          const double u = wp[i], v = wq[i];
          wp[i] = c * u - s * v;
          wq[i] = s * u + c * v;
        }
      }
      __syncthreads();
    }
    if (gl == 0) off_g[grp] = offmax;
    __syncthreads();
    if (tid == 0) {
      double mx = 0.0;
      for (int w = 0; w < NGRP; ++w) mx = fmax(mx, off_g[w]);
      done = (mx <= tol) ? 1 : 0;
    }
    __syncthreads();
    if (tid == 0 && sweep_count) atomicAdd(sweep_count, 1ULL);
    if (done) break;
  }
  jacobi_emit(X, ldx, W, ldw, m, n, colnorm, perm, b, U, ldu, sU, S, sS, V, ldv, sV);
}

// ---------------------------------------------------------------------------
// The same one-sided Jacobi SVD for m, n <= 128 with the work matrix and the
// rotation accumulator in LDS, organised for round latency: columns are
// zero-padded to a multiple of 16 rows (so a 16-lane group reads a column
// with unmasked loads), each group loads its pair of X and W columns at
// once, the three dot products are reduced inside the group with row
// rotations (DPP, no LDS round trip; every lane ends with the same sum), and
// the round-robin pairing advances by increments instead of divisions.  One
// barrier per round.  Results are those of jacobi_svd_kernel up to rounding.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ inline double dpp_row(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// sum over the 16 lanes of a row by rotations of 8, 4, 2, 1 lanes
__device__ inline double row_sum16(double v) {
  v += dpp_row<0x128>(v);
  v += dpp_row<0x124>(v);
  v += dpp_row<0x122>(v);
  v += dpp_row<0x121>(v);
  return v;
}

constexpr int JF_MAX = 8;  // 16-row slices per column: m, n <= 128

// ME, NE: 16-row slices of the X and W columns (compile-time, so that a
// lane's loads, dot products and rotations are straight-line code)
template <int ME, int NE>
__global__ __launch_bounds__(1024) void jacobi_svd_fast_kernel(
    const double* __restrict__ Ain, int lda, long long sA, double* __restrict__ U, int ldu,
    long long sU, double* __restrict__ S, long long sS, double* __restrict__ V, int ldv,
    long long sV, int m, int n, int max_sweeps, double tol,
    unsigned long long* __restrict__ sweep_count) {
  extern __shared__ double lds[];
  const long long b = blockIdx.x;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const double* A = Ain + b * sA;
  constexpr int ldx = 16 * ME + 1, ldw = 16 * NE + 1;  // odd strides
  double* X = lds;                                    // X[j * ldx + i], rows >= m zero
  double* W = lds + (size_t)ldx * n;                  // W[j * ldw + i], rows >= n zero
  __shared__ double colnorm[128];
  __shared__ int perm[128];
  __shared__ int rot_g[64];
  __shared__ int done;
  for (int t = tid; t < ldx * n; t += nthr) {
    const int j = t / ldx, i = t % ldx;
    X[t] = i < m ? A[(long long)i * lda + j] : 0.0;
  }
  for (int t = tid; t < ldw * n; t += nthr) {
    const int j = t / ldw, i = t % ldw;
    W[t] = i == j ? 1.0 : 0.0;
  }
  if (tid == 0) done = 0;
  __syncthreads();
  const int grp = tid >> 4, gl = tid & 15;
  const int N = (n + 1) & ~1;  // players incl. a dummy when n is odd
  const bool active = grp < N / 2;
  // round r pairs player 0 (group 0 only) or 1 + (grp - 1 + r) mod (N - 1)
  // with 1 + (N - 2 - grp + r) mod (N - 1)
  int u = grp >= 1 ? grp - 1 : 0, v = N - 2 - grp;
  for (int sweep = 0; sweep < max_sweeps && n > 1; ++sweep) {
    // a sweep with no rotation ends the iteration: every pair is then
    // orthogonal to tol
    int rotated = 0;
    for (int r = 0; r < N - 1; ++r) {
      if (active) {
        const int p0 = grp == 0 ? 0 : 1 + u, p1 = 1 + v;
        if (p0 < n && p1 < n) {
          const int p = min(p0, p1), q = max(p0, p1);
          double* xp = X + p * ldx + gl;
          double* xq = X + q * ldx + gl;
          double xu[ME], xv[ME];
#pragma unroll
          for (int e = 0; e < ME; ++e) {
            xu[e] = xp[16 * e];
            xv[e] = xq[16 * e];
          }
          double a = 0.0, bb = 0.0, g = 0.0;
#pragma unroll
          for (int e = 0; e < ME; ++e) {
            a += xu[e] * xu[e];
            bb += xv[e] * xv[e];
            g += xu[e] * xv[e];
          }
          a = row_sum16(a);
          bb = row_sum16(bb);
          g = row_sum16(g);
          const double scale = sqrt(a * bb);
          if (scale != 0.0 && fabs(g) > tol * scale) {
            rotated = 1;
            const double z = (bb - a) / (2.0 * g);
            const double t = (z >= 0.0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
            const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
#pragma unroll
            for (int e = 0; e < ME; ++e) {
              xp[16 * e] = c * xu[e] - sn * xv[e];
              xq[16 * e] = sn * xu[e] + c * xv[e];
            }
            // the accumulator columns only for pairs that rotate
            double* wp = W + p * ldw + gl;
            double* wq = W + q * ldw + gl;
            double wu[NE], wv[NE];
#pragma unroll
            for (int e = 0; e < NE; ++e) {
              wu[e] = wp[16 * e];
              wv[e] = wq[16 * e];
            }
#pragma unroll
            for (int e = 0; e < NE; ++e) {
              wp[16 * e] = c * wu[e] - sn * wv[e];
              wq[16 * e] = sn * wu[e] + c * wv[e];
            }
          }
        }
        u = u + 1 == N - 1 ? 0 : u + 1;
        v = v + 1 == N - 1 ? 0 : v + 1;
      }
      __syncthreads();
    }
    if (gl == 0 && active) rot_g[grp] = rotated;
    __syncthreads();
    if (tid == 0) {
      int any = 0;
      for (int w = 0; w < N / 2; ++w) any |= rot_g[w];
      done = any ? 0 : 1;
      if (sweep_count) atomicAdd(sweep_count, 1ULL);
    }
    __syncthreads();
    if (done) break;
  }
  jacobi_emit(X, ldx, W, ldw, m, n, colnorm, perm, b, U, ldu, sU, S, sS, V, ldv, sV);
}

typedef void (*jacobi_fast_fn)(const double*, int, long long, double*, int, long long, double*,
                               long long, double*, int, long long, int, int, int, double,
                               unsigned long long*);

#define TN_JF_ROW(ME)                                                                          \
  {jacobi_svd_fast_kernel<ME, 1>, jacobi_svd_fast_kernel<ME, (ME >= 2 ? 2 : ME)>,              \
   jacobi_svd_fast_kernel<ME, (ME >= 3 ? 3 : ME)>, jacobi_svd_fast_kernel<ME, (ME >= 4 ? 4 : ME)>, \
   jacobi_svd_fast_kernel<ME, (ME >= 5 ? 5 : ME)>, jacobi_svd_fast_kernel<ME, (ME >= 6 ? 6 : ME)>, \
   jacobi_svd_fast_kernel<ME, (ME >= 7 ? 7 : ME)>, jacobi_svd_fast_kernel<ME, (ME >= 8 ? 8 : ME)>}

// the kernel for me, ne slices (1 <= ne <= me <= JF_MAX)
jacobi_fast_fn jacobi_fast_kernel(int me, int ne) {
  static const jacobi_fast_fn table[JF_MAX][JF_MAX] = {TN_JF_ROW(1), TN_JF_ROW(2), TN_JF_ROW(3),
                                                      TN_JF_ROW(4), TN_JF_ROW(5), TN_JF_ROW(6),
                                                      TN_JF_ROW(7), TN_JF_ROW(8)};
  return table[me - 1][ne - 1];
}
#undef TN_JF_ROW

// ---------------------------------------------------------------------------
// One-sided Jacobi SVD of one large matrix (n <= 512) across the whole GPU:
// the work matrix and the rotation accumulator live in global memory as
// contiguous columns, and each launch is one round of the round-robin
// ordering with one workgroup per column pair.  The largest relative
// off-diagonal of a sweep is collected with an atomic maximum on the bit
// pattern (order-preserving for non-negative doubles).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void jacobi_round_kernel(double* __restrict__ X, int ldx,
                                                           double* __restrict__ W, int ldw, int m,
                                                           int n, int N, int r, double tol,
                                                           const double* __restrict__ null2,
                                                           unsigned long long* __restrict__ offbits) {
  __shared__ double red[3][4];
  const int q = blockIdx.x;
  const int p0 = q == 0 ? 0 : 1 + (q - 1 + r) % (N - 1);
  const int p1 = 1 + (N - 2 - q + r) % (N - 1);
  if (p0 >= n || p1 >= n) return;
  const int p = min(p0, p1), qq = max(p0, p1);
  double* xp = X + (long long)p * ldx;
  double* xq = X + (long long)qq * ldx;
  // columns of up to 512 rows stay in registers between the dot products
  // and the rotation (two entries per thread)
  const bool held = m <= 512;
  double us[2] = {0.0, 0.0}, vs[2] = {0.0, 0.0};
  double a = 0.0, bb = 0.0, g = 0.0;
  if (held) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int i = threadIdx.x + 256 * k;
      if (i < m) {
        us[k] = xp[i];
        vs[k] = xq[i];
        a += us[k] * us[k];
        bb += vs[k] * vs[k];
        g += us[k] * vs[k];
      }
    }
  } else {
    for (int i = threadIdx.x; i < m; i += 256) {
      const double u = xp[i], v = xq[i];
      a += u * u;
      bb += v * v;
      g += u * v;
    }
  }
  // the three sums in one exchange: each a wave sum, then the four wave
  // partials in order
  a = wave_sum(a);
  bb = wave_sum(bb);
  g = wave_sum(g);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = bb;
    red[2][threadIdx.x >> 6] = g;
  }
  __syncthreads();
  a = red[0][0] + red[0][1] + red[0][2] + red[0][3];
  bb = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  g = red[2][0] + red[2][1] + red[2][2] + red[2][3];
  // a numerically null column (squared norm at most null2) is left alone:
  // its direction is rounding noise, and rotating it never settles
  if (a <= null2[0] || bb <= null2[0]) return;
  const double scale = sqrt(a * bb);
  if (scale == 0.0 || fabs(g) <= tol * scale) return;
  if (threadIdx.x == 0)
    atomicMax(offbits, (unsigned long long)__double_as_longlong(fabs(g) / scale));
  const double z = (bb - a) / (2.0 * g);
  const double t = (z >= 0.0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
  const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
  if (held) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int i = threadIdx.x + 256 * k;
      if (i < m) {
        xp[i] = c * us[k] - sn * vs[k];
        xq[i] = sn * us[k] + c * vs[k];
      }
    }
  } else {
    for (int i = threadIdx.x; i < m; i += 256) {
      const double u = xp[i], v = xq[i];
      xp[i] = c * u - sn * v;
      xq[i] = sn * u + c * v;
    }
  }
  double* wp = W + (long long)p * ldw;
  double* wq = W + (long long)qq * ldw;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double u = wp[i], v = wq[i];
    wp[i] = c * u - sn * v;
    wq[i] = sn * u + c * v;
  }
}

// out[0] = scale2 * sum x^2 over n entries, in one workgroup (a fixed order)
__global__ __launch_bounds__(1024) void sumsq_kernel(const double* __restrict__ x, long long n,
                                                     double scale2, double* __restrict__ out) {
  __shared__ double red[16];
  double a = 0.0;
  for (long long i = threadIdx.x; i < n; i += 1024) a += x[i] * x[i];
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w];
    out[0] = scale2 * t;
  }
}

// dst[i][c0 + j] = src[i][j] for an m x nc block (row-major, leading dims)
__global__ void copy_cols_kernel(const double* __restrict__ src, int lds, double* __restrict__ dst,
                                 int ldd, int m, int nc) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)m * nc) return;
  const int i = (int)(t / nc), j = (int)(t % nc);
  dst[(long long)i * ldd + j] = src[(long long)i * lds + j];
}

// Householder QR on column-contiguous storage Xq[c][r] (row c of Xq is
// column c of the matrix, length m).  Reflector j: from x = Xq[j][j..m),
// beta = -sign(x_j) |x|, v = (1, x_{j+1..} / (x_j - beta)), tau = (beta -
// x_j) / beta; on exit Xq[j][j] = beta (the diagonal of R), Xq[j][r > j] the
// tail of v, tau[j] (0 when the tail is zero: H = I).
__global__ __launch_bounds__(256) void hh_vec_kernel(double* __restrict__ Xq, int ld, int m,
                                                     int j, double* __restrict__ tau) {
  __shared__ double red[4];
  double* x = Xq + (long long)j * ld;
  const double alpha = x[j];  // read by every thread before thread 0 rewrites it
  double a = 0.0;
  for (int r = j + 1 + threadIdx.x; r < m; r += 256) a += x[r] * x[r];
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  const double xn2 = red[0] + red[1] + red[2] + red[3];
  if (xn2 == 0.0) {
    if (threadIdx.x == 0) tau[j] = 0.0;
    return;
  }
  const double beta = alpha >= 0.0 ? -sqrt(alpha * alpha + xn2) : sqrt(alpha * alpha + xn2);
  const double sc = 1.0 / (alpha - beta);
  for (int r = j + 1 + threadIdx.x; r < m; r += 256) x[r] *= sc;
  if (threadIdx.x == 0) {
    x[j] = beta;
    tau[j] = (beta - alpha) / beta;
  }
}

// y <- (I - tau v v^T) y for the columns c = c0 + blockIdx.x of Y (column-
// contiguous, rows j..m of each touched), v = (1, Xq[j][j+1..m)).
__global__ __launch_bounds__(256) void hh_apply_kernel(const double* __restrict__ Xq, int ldq,
                                                       double* __restrict__ Y, int ldy, int m,
                                                       int j, const double* __restrict__ tau,
                                                       int c0) {
  __shared__ double red[4];
  const double t = tau[j];
  if (t == 0.0) return;
  const double* v = Xq + (long long)j * ldq;
  double* y = Y + (long long)(c0 + blockIdx.x) * ldy;
  double a = threadIdx.x == 0 ? y[j] : 0.0;
  for (int r = j + 1 + threadIdx.x; r < m; r += 256) a += v[r] * y[r];
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  const double sdot = t * (red[0] + red[1] + red[2] + red[3]);
  if (threadIdx.x == 0) y[j] -= sdot;
  for (int r = j + 1 + threadIdx.x; r < m; r += 256) y[r] -= sdot * v[r];
}

// dst[r][c] = src[c][r] for a rows x cols destination (leading dimensions
// ldd, lds)
__global__ void transpose_kernel(const double* __restrict__ src, int lds, double* __restrict__ dst,
                                 int ldd, int rows, int cols) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)rows * cols) return;
  const int r = (int)(t / cols), c = (int)(t % cols);
  dst[(long long)r * ldd + c] = src[(long long)c * lds + r];
}

// dst[r][c] = src[r][c] for c <= r, 0 above (n x n)
__global__ void lower_copy_kernel(const double* __restrict__ src, int lds, double* __restrict__ dst,
                                  int ldd, int n) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * n) return;
  const int r = (int)(t / n), c = (int)(t % n);
  dst[(long long)r * ldd + c] = c <= r ? src[(long long)r * lds + c] : 0.0;
}

// X[j][i] = A[i][j] (columns contiguous), W = I
__global__ void jacobi_setup_kernel(const double* __restrict__ A, int lda, int m, int n,
                                    double* __restrict__ X, double* __restrict__ W) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < (long long)m * n) {
    const int j = (int)(t / m), i = (int)(t % m);
    X[t] = A[(long long)i * lda + j];
  }
  if (t < (long long)n * n) {
    const int j = (int)(t / n), i = (int)(t % n);
    W[t] = i == j ? 1.0 : 0.0;
  }
}

__global__ __launch_bounds__(1024) void jacobi_emit_kernel(const double* X, int ldx,
                                                           const double* W, int ldw, int m, int n,
                                                           double* __restrict__ U, int ldu,
                                                           double* __restrict__ S,
                                                           double* __restrict__ V, int ldv) {
  __shared__ double colnorm[512];
  __shared__ int perm[512];
  jacobi_emit(X, ldx, W, ldw, m, n, colnorm, perm, 0, U, ldu, 0, S, 0, V, ldv, 0);
}

// ---------------------------------------------------------------------------
// Cholesky of G + shift I and the inverse of its upper factor.  The trailing
// matrix lives in LDS; step j reads the unscaled row j, writes row j of R
// (divided by sqrt of the pivot) and updates the trailing block with
// W[r][c] -= W[j][r] W[j][c] / W[j][j] -- one barrier per step.  The inverse
// is a column-oriented back substitution over all columns at once, also one
// barrier per step, reading R from LDS when it fits there too.
// ---------------------------------------------------------------------------
constexpr int CHOL_THREADS = 1024;

// R_IN_LDS: the rows of R are kept in LDS too (compile-time, see above).
// W_IN_LDS false: the trailing matrix lives in the Rinv output instead (for
// k whose k x k block does not fit in LDS; it becomes R^-1 in place), and R
// in the R output; the barriers order these global accesses within the
// workgroup.
template <bool R_IN_LDS, bool W_IN_LDS = true>
__global__ __launch_bounds__(CHOL_THREADS) void cholesky_inv_kernel(
    const double* __restrict__ G, int k, double shift_rel, double* __restrict__ R,
    double* __restrict__ Rinv, int* __restrict__ info) {
  extern __shared__ double lds[];
  {
    const long long off = (long long)blockIdx.x * k * k;  // one matrix per workgroup
    G += off;
    R += off;
    Rinv += off;
    info += blockIdx.x;
  }
  double* Wk = W_IN_LDS ? lds : Rinv;  // k x k trailing matrix, later R^-1
  double* Rl;  // R rows as they are produced
  if constexpr (R_IN_LDS)
    Rl = lds + k * k;
  else
    Rl = R;
  const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5;
  __shared__ double shift;
  if (tid < 64) {
    double tr = 0.0;
    for (int i = tid; i < k; i += 64) tr += G[i * k + i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) tr += __shfl_xor(tr, o, 64);
    if (tid == 0) shift = shift_rel * tr;
  }
  __syncthreads();
  for (int t = tid; t < k * k; t += CHOL_THREADS) {
    const int i = t / k, j = t % k;
    Wk[t] = G[t] + ((i == j) ? shift : 0.0);
    Rl[t] = 0.0;
  }
  __syncthreads();
  int fail = 0;
  for (int j = 0; j < k; ++j) {
    const double dj = Wk[j * k + j];
    if (!(dj > 0.0)) {  // every thread sees the same pivot
      fail = j + 1;
      break;
    }
    const double inv_d = 1.0 / dj, inv_r = 1.0 / sqrt(dj);
    for (int c = j + tid; c < k; c += CHOL_THREADS) Rl[j * k + c] = Wk[j * k + c] * inv_r;
    // trailing update of the upper triangle, rows over ty, columns over tx
    for (int r = j + 1 + ty; r < k; r += 32) {
      const double wr = Wk[j * k + r] * inv_d;
      for (int c = r + tx; c < k; c += 32) Wk[r * k + c] -= wr * Wk[j * k + c];
    }
    __syncthreads();
  }
  if (tid == 0) *info = fail;
  if (fail) return;
  // R^-1 by column-oriented back substitution on all columns at once (Wk is
  // free): B = I; for j = k-1 .. 0, with row j of B final,
  // B[i][c] -= R[i][j] B[j][c] / R[j][j] for i < j <= c; finally row j of
  // R^-1 is B[j][:] / R[j][j].  One barrier per step; the work of a step is
  // spread over all threads.
  for (int t = tid; t < k * k; t += CHOL_THREADS) Wk[t] = (t / k == t % k) ? 1.0 : 0.0;
  __syncthreads();
  for (int j = k - 1; j > 0; --j) {
    const double inv_jj = 1.0 / Rl[j * k + j];
    const int w = k - j;
    for (int t = tid; t < j * w; t += CHOL_THREADS) {
      const int i = t / w, c = j + t % w;
      Wk[i * k + c] -= Rl[i * k + j] * (Wk[j * k + c] * inv_jj);
    }
    __syncthreads();
  }
  for (int t = tid; t < k * k; t += CHOL_THREADS) {
    const int i = t / k;
    Rinv[t] = Wk[t] / Rl[i * k + i];  // in place when Wk is Rinv
    if constexpr (R_IN_LDS) R[t] = Rl[t];
  }
}

// ---------------------------------------------------------------------------
// The same factorisation and inverse for k <= 128 with the trailing matrix in
// registers: thread (ty, tx) of a 32 x 32 grid holds the entries of rows
// ty + 32a and columns tx + 32b (a, b < 4).  Cholesky step j: the 32 threads
// holding row j scale it by 1/sqrt(pivot) and publish it as row j of R in
// LDS; after one barrier every thread applies W[r][c] -= R[j][r] R[j][c] to
// its 16 entries (entries of finished rows and columns are updated too and
// never read again).  The same row operations carried on an identity block
// give R^-T in the same k steps (Gauss-Jordan on [G | I]), so the inverse
// costs no second sweep.  One barrier per step.
// ---------------------------------------------------------------------------
constexpr int CHOLR_MAX = 128;

__device__ inline double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__global__ __launch_bounds__(1024) void cholesky_inv_reg_kernel(const double* __restrict__ G, int k,
                                                                double shift_rel,
                                                                double* __restrict__ R,
                                                                double* __restrict__ Rinv,
                                                                int* __restrict__ info) {
  extern __shared__ double lds[];
  {
    const long long off = (long long)blockIdx.x * k * k;  // one matrix per workgroup
    G += off;
    R += off;
    Rinv += off;
    info += blockIdx.x;
  }
  const int ldr = k | 1;
  double* Rl = lds;                      // R, row j at Rl + j * ldr
  double* xrow = lds + (size_t)k * ldr;  // [2][CHOLR_MAX], rows of X in flight
  double* piv = xrow + 2 * CHOLR_MAX;    // [CHOLR_MAX], pivot of each step
  const int tid = threadIdx.x, ty = tid >> 5, tx = tid & 31;
  __shared__ double shift;
  if (tid < 64) {
    double tr = 0.0;
    for (int i = tid; i < k; i += 64) tr += G[i * k + i];
    tr = wave_sum(tr);
    if (tid == 0) shift = shift_rel * tr;
  }
  for (int t = tid; t < k * ldr; t += 1024) Rl[t] = 0.0;
  __syncthreads();
  // The elimination runs on [G | I]: row operations that take G to R take
  // the identity to R^-T, so the inverse comes out of the same sweep.
  // Thread (ty, tx) holds G entries and identity entries (ty + 32 a,
  // tx + 32 b).
  double W[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int r = ty + 32 * a, c = tx + 32 * b;
      W[a][b] = (r < k && c < k) ? G[r * k + c] + (r == c ? shift : 0.0) : 0.0;
    }
  // A Gram matrix within 1e-9 of the identity (the second pass of
  // Cholesky-QR on a block that is already orthonormal): with E = G - I,
  // R = I + U and R^-1 = I - U, U the strict upper part of E plus half its
  // diagonal; the neglected terms are below k max|E|^2 <= 1.3e-16.
  // (a NaN anywhere propagates into the maximum and sends the matrix down
  // the elimination, which reports it as a failed pivot)
  auto nan_max = [](double x, double y) { return (y > x || y != y) ? y : x; };
  __shared__ double emax_w[16];
  {
    double em = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int r = ty + 32 * a, c = tx + 32 * b;
        if (r < k && c < k) em = nan_max(em, fabs(W[a][b] - (r == c ? 1.0 : 0.0)));
      }
    for (int o = 32; o > 0; o >>= 1) em = nan_max(em, __shfl_xor(em, o, 64));
    if ((tid & 63) == 0) emax_w[tid >> 6] = em;
  }
  __syncthreads();
  double emax = 0.0;
  for (int w = 0; w < 16; ++w) emax = nan_max(emax, emax_w[w]);
  if (shift == 0.0 && emax <= 1e-9) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int r = ty + 32 * a, c = tx + 32 * b;
        if (r < k && c < k) {
          const double e = W[a][b] - (r == c ? 1.0 : 0.0);
          const double u = r < c ? e : (r == c ? 0.5 * e : 0.0);
          R[r * k + c] = (r == c ? 1.0 : 0.0) + u;
          Rinv[r * k + c] = (r == c ? 1.0 : 0.0) - u;
        }
      }
    if (tid == 0) *info = 0;
    return;
  }
  double Z[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) Z[a][b] = ty + 32 * a == tx + 32 * b ? 1.0 : 0.0;
  // Step j: the holders of row j scale it by 1 / sqrt(pivot), which gives
  // row j of R and row j of R^-T (column j of R^-1); every row i then takes
  // R[j][i] times those rows (row j itself drops to zero).  A failing pivot
  // (not positive) zeroes its rows and the elimination runs on to the end;
  // the first failure is reported afterwards, so no step waits on a status
  // read.  One barrier per step: the R^-T rows in flight are double-buffered.
#pragma unroll
  for (int jb = 0; jb < 4; ++jb) {
    for (int jj = 0; jj < 32; ++jj) {
      const int j = 32 * jb + jj;
      if (j >= k) break;
      double* xr = xrow + (j & 1) * CHOLR_MAX;
      if (ty == jj) {
        // the pivot W[j][j] sits in lane 32 (jj & 1) + jj of this wave
        const double d = readlane_d(W[jb][jb], ((jj & 1) << 5) + jj);
        const double ir = d > 0.0 ? rsqrt(d) : 0.0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int c = tx + 32 * b;
          if (c < k) {
            const double v = c >= j ? W[jb][b] * ir : 0.0;
            Rl[j * ldr + c] = v;
            R[j * k + c] = v;
            const double x = c <= j ? Z[jb][b] * ir : 0.0;
            xr[c] = x;
            Rinv[c * k + j] = x;
          }
        }
        if (tx == 0) piv[j] = d;
      }
      __syncthreads();
      double rr[4], rc[4], xc[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) rr[a] = ty + 32 * a < k ? Rl[j * ldr + ty + 32 * a] : 0.0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        rc[b] = tx + 32 * b < k ? Rl[j * ldr + tx + 32 * b] : 0.0;
        xc[b] = tx + 32 * b < k ? xr[tx + 32 * b] : 0.0;
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          W[a][b] -= rr[a] * rc[b];
          Z[a][b] -= rr[a] * xc[b];
        }
    }
  }
  if (tid < 64) {
    int f = 0x7fffffff;
    for (int j = tid; j < k; j += 64)
      if (!(piv[j] > 0.0)) f = min(f, j + 1);
    for (int o = 32; o > 0; o >>= 1) f = min(f, __shfl_xor(f, o, 64));
    if (tid == 0) *info = f == 0x7fffffff ? 0 : f;
  }
}

__global__ void scale_columns_kernel(int m, int n, double* X, int ldx, const double* s,
                                     int invsqrt, double cut) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)m * n) return;
  const int i = (int)(t / n), j = (int)(t % n);
  double f = s[j];
  if (invsqrt) f = (f > cut * s[0]) ? 1.0 / sqrt(f) : 0.0;
  X[(long long)i * ldx + j] *= f;
}

// dst = src / ||src||_F in one workgroup (small tensors); a zero tensor is
// copied unchanged
__global__ __launch_bounds__(1024) void frob_normalize_kernel(const double* src, double* dst,
                                                              long long n, double* norm_out) {
  __shared__ double part[16];
  double a = 0.0;
  for (long long i = threadIdx.x; i < n; i += 1024) a += src[i] * src[i];
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < 16; ++w) s += part[w];
    part[0] = sqrt(s);
    if (norm_out) *norm_out = part[0];
  }
  __syncthreads();
  const double nrm = part[0];
  const double inv = nrm > 0.0 ? 1.0 / nrm : 1.0;
  for (long long i = threadIdx.x; i < n; i += 1024) dst[i] = src[i] * inv;
}

// The same for large tensors over many workgroups: per-workgroup sums of
// squares, then every workgroup of the scaling pass adds them up in the same
// order (so all use the same norm) and scales its part.
constexpr int FROB_BLOCKS = 256;

__global__ __launch_bounds__(256) void frob_partial_kernel(const double* src, long long n,
                                                           double* part) {
  __shared__ double red[4];
  double a = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    a += src[i] * src[i];
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void frob_scale_kernel(const double* src, double* dst,
                                                         long long n, const double* part,
                                                         int nparts, double* norm_out) {
  __shared__ double inv;
  if (threadIdx.x < 64) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 64) s += part[i];
    s = wave_sum(s);
    if (threadIdx.x == 0) {
      const double nrm = sqrt(s);
      inv = nrm > 0.0 ? 1.0 / nrm : 1.0;
      if (norm_out && blockIdx.x == 0) *norm_out = nrm;
    }
  }
  __syncthreads();
  const double f = inv;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    dst[i] = src[i] * f;
}

// splitmix64 (Steele, Lea, Flood 2014) mapped to a uniform value in [-1, 1)
__global__ void fill_random_kernel(double* x, long long n, unsigned long long seed) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  unsigned long long z = seed + 0x9E3779B97F4A7C15ULL * (unsigned long long)(i + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z = z ^ (z >> 31);
  x[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

constexpr size_t LDS_LIMIT = 150 * 1024;

}  // namespace

// device-side sweep counter for diagnostics (read by tn_prof_read)
__device__ unsigned long long g_sweep_counter = 0;
static unsigned long long* g_sweeps = nullptr;

int jacobi_sweeps_read(tn_ctx* ctx, unsigned long long* out) {
  if (!g_sweeps) TN_HIP(ctx, hipGetSymbolAddress((void**)&g_sweeps, HIP_SYMBOL(g_sweep_counter)));
  TN_HIP(ctx, hipMemcpy(out, g_sweeps, sizeof(unsigned long long), hipMemcpyDeviceToHost));
  const unsigned long long zero = 0;
  TN_HIP(ctx, hipMemcpy(g_sweeps, &zero, sizeof(zero), hipMemcpyHostToDevice));
  return TN_OK;
}

bool jacobi_svd_needs_workspace(int m, int n) {
  const int me = (m + 15) / 16, ne = (n + 15) / 16;
  const size_t fast_bytes = (size_t)(16 * me + 1 + 16 * ne + 1) * n * sizeof(double);
  if (m <= 16 * JF_MAX && fast_bytes <= LDS_LIMIT) return false;
  const size_t per = (size_t)(m | 1) * n + (size_t)(n | 1) * n;
  return per * sizeof(double) > LDS_LIMIT;
}

int side_stream_ready(tn_ctx* ctx) {
  if (ctx->side) return TN_OK;
  TN_HIP(ctx, hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
  TN_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
  TN_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
  return TN_OK;
}

int jacobi_svd(tn_ctx* ctx, int batch, int m, int n, double* A, int lda, long long sA, double* U,
               int ldu, long long sU, double* S, long long sS, double* V, int ldv, long long sV) {
  if (m < n) TN_FAIL(ctx, TN_EINVAL, "jacobi_svd needs m >= n (m=%d n=%d)", m, n);
  if (n > 512) TN_FAIL(ctx, TN_EINVAL, "jacobi_svd supports n <= 512 (n=%d)", n);
  if (batch <= 0 || n <= 0) return TN_OK;
  if (!g_sweeps) TN_HIP(ctx, hipGetSymbolAddress((void**)&g_sweeps, HIP_SYMBOL(g_sweep_counter)));
  const size_t mark = ctx->arena_off;  // stream order makes the slice reusable afterwards
  const size_t per = (size_t)(m | 1) * n + (size_t)(n | 1) * n;  // padded columns
  const size_t lds_bytes = per * sizeof(double);
  double* work = nullptr;
  size_t dyn = 0;
  if (lds_bytes <= LDS_LIMIT) {
    dyn = lds_bytes;
  } else {
    work = ws_alloc<double>(ctx, (size_t)batch * per);
    if (!work) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted in jacobi_svd");
  }
  // rotations stop once every column pair is orthogonal to the rounding
  // level of its dot product (about m ulp), or the sweeps would never end
  const double tol = 8.0 * 1.1102230246251565e-16 * (double)m;
  {
    const int me = (m + 15) / 16, ne = (n + 15) / 16;
    const size_t fast_bytes = (size_t)(16 * me + 1 + 16 * ne + 1) * n * sizeof(double);
    if (m <= 16 * JF_MAX && fast_bytes <= LDS_LIMIT) {
      const int groups = ((n + 1) & ~1) / 2;
      const unsigned threads = (unsigned)std::max(64, (16 * groups + 63) / 64 * 64);
      hipLaunchKernelGGL(jacobi_fast_kernel(me, ne), dim3(batch), dim3(threads), fast_bytes,
                         ctx->stream, A, lda, sA, U, ldu, sU, S, sS, V, ldv, sV, m, n, 80, tol,
                         g_sweeps);
      TN_HIP(ctx, hipGetLastError());
      return TN_OK;
    }
  }
  if (work)
    hipLaunchKernelGGL(jacobi_svd_kernel<true>, dim3(batch), dim3(SVD_THREADS), dyn, ctx->stream,
                       A, lda, sA, U, ldu, sU, S, sS, V, ldv, sV, m, n, work, 80, tol, g_sweeps);
  else
    hipLaunchKernelGGL(jacobi_svd_kernel<false>, dim3(batch), dim3(SVD_THREADS), dyn, ctx->stream,
                       A, lda, sA, U, ldu, sU, S, sS, V, ldv, sV, m, n, work, 80, tol, g_sweeps);
  TN_HIP(ctx, hipGetLastError());
  ctx->arena_off = mark;
  return TN_OK;
}

// Columns m x nc of Z orthonormal and orthogonal to the first r columns of
// U (m x r, orthonormal, leading dimension ldu): a seeded random start,
// projected off U_r twice, then two Cholesky-QR passes; written into
// U[:, r : r + nc].
// SVD of one m x n matrix (m >= n, n <= 512) with a QR preconditioner:
// A = Q R by Householder reflections (on column-contiguous storage), then
// the one-sided Jacobi SVD of R^T = U' S W^T (jacobi_svd_large), so that
// A = (Q W) S U'^T.  On a graded matrix the Jacobi sweeps on R^T are far
// fewer than on A itself.
int svd_qr_large(tn_ctx* ctx, int m, int n, const double* A, int lda, double* U, int ldu,
                 double* S, double* V, int ldv) {
  if (m < n || n < 1 || n > 512) TN_FAIL(ctx, TN_EINVAL, "svd_qr_large needs 1 <= n <= m, n <= 512");
  const size_t mark = ctx->arena_off;
  double* Xq = ws_alloc<double>(ctx, (size_t)n * m);   // [n][m]: column c of A
  double* Rt = ws_alloc<double>(ctx, (size_t)n * n);   // R^T, row-major
  double* Ue = ws_alloc<double>(ctx, (size_t)n * n);
  double* We = ws_alloc<double>(ctx, (size_t)n * n);
  double* Y = ws_alloc<double>(ctx, (size_t)n * m);    // [n][m]: columns of Q W
  double* tau = ws_alloc<double>(ctx, (size_t)n);
  if (!tau) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted in svd_qr_large");
  const long long nm = (long long)n * m, nn = (long long)n * n;
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)((nm + 255) / 256)), dim3(256), 0,
                     ctx->stream, A, lda, Xq, m, n, m);
  TN_HIP(ctx, hipGetLastError());
  for (int j = 0; j < n; ++j) {
    hipLaunchKernelGGL(hh_vec_kernel, dim3(1), dim3(256), 0, ctx->stream, Xq, m, m, j, tau);
    if (j + 1 < n)
      hipLaunchKernelGGL(hh_apply_kernel, dim3((unsigned)(n - j - 1)), dim3(256), 0, ctx->stream,
                         Xq, m, Xq, m, m, j, tau, j + 1);
  }
  TN_HIP(ctx, hipGetLastError());
  // R^T[i][c] = R[c][i] = Xq[i][c] for c <= i, zero above
  hipLaunchKernelGGL(lower_copy_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0,
                     ctx->stream, Xq, m, Rt, n, n);
  TN_HIP(ctx, hipGetLastError());
  TN_TRY(jacobi_svd_large(ctx, n, n, Rt, n, Ue, n, S, We, n));
  // Q W: the columns of W (length n) padded to m, the reflectors applied
  // in reverse order
  TN_HIP(ctx, hipMemsetAsync(Y, 0, (size_t)nm * sizeof(double), ctx->stream));
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0,
                     ctx->stream, We, n, Y, m, n, n);
  TN_HIP(ctx, hipGetLastError());
  for (int j = n - 1; j >= 0; --j)
    hipLaunchKernelGGL(hh_apply_kernel, dim3((unsigned)n), dim3(256), 0, ctx->stream, Xq, m, Y, m,
                       m, j, tau, 0);
  TN_HIP(ctx, hipGetLastError());
  // U[r][i] = (Q W)[r][i] = Y[i][r]; V = U'
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)((nm + 255) / 256)), dim3(256), 0,
                     ctx->stream, Y, m, U, ldu, m, n);
  hipLaunchKernelGGL(copy_cols_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0,
                     ctx->stream, Ue, n, V, ldv, n, n);
  TN_HIP(ctx, hipGetLastError());
  ctx->arena_off = mark;
  return TN_OK;
}

static int complete_left_basis(tn_ctx* ctx, int m, int r, int nc, double* U, int ldu) {
  if (nc <= 0) return TN_OK;
  const size_t mark = ctx->arena_off;
  double* Z = ws_alloc<double>(ctx, (size_t)m * nc);
  double* Z2 = ws_alloc<double>(ctx, (size_t)m * nc);
  double* T = ws_alloc<double>(ctx, (size_t)std::max(r, 1) * nc);
  double* G = ws_alloc<double>(ctx, (size_t)nc * nc);
  double* R = ws_alloc<double>(ctx, (size_t)nc * nc);
  double* Ri = ws_alloc<double>(ctx, (size_t)nc * nc);
  int* info = ws_alloc<int>(ctx, 2);
  if (!info) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted completing the left basis");
  TN_TRY(fill_random(ctx, Z, (long long)m * nc, 0x6a09e667f3bcc909ULL));
  for (int pass = 0; pass < 2 && r > 0; ++pass) {
    TN_TRY(gemm(ctx, r, nc, m, U, ldu, true, Z, nc, false, T, nc, 1.0, 0.0));
    TN_TRY(gemm(ctx, m, nc, r, U, ldu, false, T, nc, false, Z, nc, -1.0, 1.0));
  }
  for (int pass = 0; pass < 2; ++pass) {
    TN_TRY(gemm(ctx, nc, nc, m, Z, nc, true, Z, nc, false, G, nc, 1.0, 0.0));
    TN_TRY(cholesky_inv(ctx, nc, G, 0.0, R, Ri, info + pass, 1));
    TN_TRY(gemm(ctx, m, nc, nc, Z, nc, false, Ri, nc, false, Z2, nc, 1.0, 0.0));
    std::swap(Z, Z2);
  }
  int hinfo[2] = {0, 0};
  TN_HIP(ctx, hipMemcpyAsync(hinfo, info, 2 * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  const long long tot = (long long)m * nc;
  hipLaunchKernelGGL(copy_cols_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                     ctx->stream, Z, nc, U + r, ldu, m, nc);
  TN_HIP(ctx, hipGetLastError());
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  ctx->arena_off = mark;
  if (hinfo[0] != 0 || hinfo[1] != 0)
    TN_FAIL(ctx, TN_ENUMERIC, "Cholesky-QR breakdown completing the left basis");
  return TN_OK;
}

int jacobi_svd_large(tn_ctx* ctx, int m, int n, const double* A, int lda, double* U, int ldu,
                     double* S, double* V, int ldv) {
  if (m < n || n < 1 || n > 512) TN_FAIL(ctx, TN_EINVAL, "jacobi_svd_large needs 1 <= n <= m, n <= 512");
  const size_t mark = ctx->arena_off;
  double* X = ws_alloc<double>(ctx, (size_t)m * n);
  double* W = ws_alloc<double>(ctx, (size_t)n * n);
  double* null2 = ws_alloc<double>(ctx, 1);
  unsigned long long* off = ws_alloc<unsigned long long>(ctx, 1);
  if (!off) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted in jacobi_svd_large");
  const long long tot = (long long)std::max(m, n) * n;
  hipLaunchKernelGGL(jacobi_setup_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                     ctx->stream, A, lda, m, n, X, W);
  TN_HIP(ctx, hipGetLastError());
  const double tol = 8.0 * 1.1102230246251565e-16 * (double)m;
  // columns with |x|^2 <= tol^2 |A|_F^2 count as numerically null
  hipLaunchKernelGGL(sumsq_kernel, dim3(1), dim3(1024), 0, ctx->stream, X, (long long)m * n,
                     tol * tol, null2);
  TN_HIP(ctx, hipGetLastError());
  const int N = (n + 1) & ~1;
  unsigned long long* hoff = reinterpret_cast<unsigned long long*>(ctx->host_scratch + 40);
  for (int sweep = 0; sweep < 80 && n > 1; ++sweep) {
    TN_HIP(ctx, hipMemsetAsync(off, 0, sizeof(unsigned long long), ctx->stream));
    for (int r = 0; r < N - 1; ++r)
      hipLaunchKernelGGL(jacobi_round_kernel, dim3(N / 2), dim3(256), 0, ctx->stream, X, m, W, n,
                         m, n, N, r, tol, null2, off);
    TN_HIP(ctx, hipGetLastError());
    TN_HIP(ctx, hipMemcpyAsync(hoff, off, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                               ctx->stream));
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (*hoff == 0) break;  // no rotation in the whole sweep
  }
  hipLaunchKernelGGL(jacobi_emit_kernel, dim3(1), dim3(1024), 0, ctx->stream, X, m, W, n, m, n, U,
                     ldu, S, V, ldv);
  TN_HIP(ctx, hipGetLastError());
  // the left vectors of the null columns (the trailing ones: S is sorted)
  // are rounding noise; replace them by an orthonormal basis of the
  // complement of the others (the right vectors, accumulated rotations,
  // are orthonormal already)
  std::vector<double> hs(n + 1);
  TN_HIP(ctx, hipMemcpyAsync(hs.data(), S, n * sizeof(double), hipMemcpyDeviceToHost,
                             ctx->stream));
  TN_HIP(ctx, hipMemcpyAsync(hs.data() + n, null2, sizeof(double), hipMemcpyDeviceToHost,
                             ctx->stream));
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  const double thr = sqrt(hs[n]);
  int r = 0;
  while (r < n && hs[r] > thr) ++r;
  TN_TRY(complete_left_basis(ctx, m, r, n - r, U, ldu));
  ctx->arena_off = mark;
  return TN_OK;
}

int cholesky_inv(tn_ctx* ctx, int k, const double* G, double shift_rel, double* R, double* Rinv,
                 int* info, int batch) {
  const size_t one = (size_t)k * k * sizeof(double);
  if (k < 1 || k > 512) TN_FAIL(ctx, TN_EINVAL, "cholesky_inv supports 1 <= k <= 512 (k=%d)", k);
  if (batch < 1) return TN_OK;
  if (one > LDS_LIMIT) {
    // the k x k block does not fit in LDS: trailing matrix and R in global
    // memory (the Rinv and R outputs)
    hipLaunchKernelGGL((cholesky_inv_kernel<false, false>), dim3(batch), dim3(CHOL_THREADS), 0,
                       ctx->stream, G, k, shift_rel, R, Rinv, info);
    TN_HIP(ctx, hipGetLastError());
    return TN_OK;
  }
  if (k <= CHOLR_MAX) {
    const size_t dyn = ((size_t)k * (k | 1) + 3 * CHOLR_MAX) * sizeof(double);
    hipLaunchKernelGGL(cholesky_inv_reg_kernel, dim3(batch), dim3(1024), dyn, ctx->stream, G, k,
                       shift_rel, R, Rinv, info);
    TN_HIP(ctx, hipGetLastError());
    return TN_OK;
  }
  const int r_in_lds = 2 * one <= LDS_LIMIT;
  if (r_in_lds)
    hipLaunchKernelGGL(cholesky_inv_kernel<true>, dim3(batch), dim3(CHOL_THREADS), 2 * one,
                       ctx->stream, G, k, shift_rel, R, Rinv, info);
  else
    hipLaunchKernelGGL(cholesky_inv_kernel<false>, dim3(batch), dim3(CHOL_THREADS), one,
                       ctx->stream, G, k, shift_rel, R, Rinv, info);
  TN_HIP(ctx, hipGetLastError());
  return TN_OK;
}

int scale_columns(tn_ctx* ctx, int m, int n, double* X, int ldx, const double* s, int invsqrt) {
  const long long tot = (long long)m * n;
  if (tot == 0) return TN_OK;
  hipLaunchKernelGGL(scale_columns_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                     ctx->stream, m, n, X, ldx, s, invsqrt, 1e-14);
  TN_HIP(ctx, hipGetLastError());
  return TN_OK;
}

int frob_normalize_to(tn_ctx* ctx, const double* src, double* dst, long long n,
                      double* norm_out) {
  if (n <= 32768) {
    hipLaunchKernelGGL(frob_normalize_kernel, dim3(1), dim3(1024), 0, ctx->stream, src, dst, n,
                       norm_out);
    TN_HIP(ctx, hipGetLastError());
    return TN_OK;
  }
  const size_t mark = ctx->arena_off;  // consumed in stream order
  double* part = ws_alloc<double>(ctx, FROB_BLOCKS);
  if (!part) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted in frob_normalize");
  const int nb = (int)std::min<long long>(FROB_BLOCKS, (n + 2047) / 2048);
  hipLaunchKernelGGL(frob_partial_kernel, dim3(nb), dim3(256), 0, ctx->stream, src, n, part);
  hipLaunchKernelGGL(frob_scale_kernel, dim3(nb), dim3(256), 0, ctx->stream, src, dst, n, part,
                     nb, norm_out);
  TN_HIP(ctx, hipGetLastError());
  ctx->arena_off = mark;
  return TN_OK;
}

int frob_normalize(tn_ctx* ctx, double* x, long long n, double* norm_out) {
  return frob_normalize_to(ctx, x, x, n, norm_out);
}

int fill_random(tn_ctx* ctx, double* x, long long n, unsigned long long seed) {
  if (n <= 0) return TN_OK;
  hipLaunchKernelGGL(fill_random_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     ctx->stream, x, n, seed);
  TN_HIP(ctx, hipGetLastError());
  return TN_OK;
}
