// Small dense FP64 linear algebra on the device: one-sided Jacobi SVD,
// Cholesky with inverse, and element-wise helpers.  One workgroup works on
// one (small) matrix; batches run as a grid of workgroups.
#include <cmath>

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
  // column norms = singular values
  for (int j = wave; j < n; j += SVD_WAVES) {
    double a = 0.0;
    for (int i = lane; i < m; i += 64) a += X[(long long)j * ldx + i] * X[(long long)j * ldx + i];
    a = wave_sum(a);
    if (lane == 0) colnorm[j] = sqrt(a);
  }
  __syncthreads();
  // rank sort, descending, ties by index
  for (int j = tid; j < n; j += SVD_THREADS) {
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
  for (int r = wave; r < n; r += SVD_WAVES) {
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

// ---------------------------------------------------------------------------
// Cholesky of G + shift I and the inverse of its upper factor.  The trailing
// matrix lives in LDS; step j reads the unscaled row j, writes row j of R
// (divided by sqrt of the pivot) and updates the trailing block with
// W[r][c] -= W[j][r] W[j][c] / W[j][j] -- one barrier per step.  The inverse
// is a column-oriented back substitution over all columns at once, also one
// barrier per step, reading R from LDS when it fits there too.
// ---------------------------------------------------------------------------
constexpr int CHOL_THREADS = 1024;

// R_IN_LDS: the rows of R are kept in LDS too (compile-time, see above)
template <bool R_IN_LDS>
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
  double* Wk = lds;                        // k x k trailing matrix, later R^-1
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
    Rinv[t] = Wk[t] / Rl[i * k + i];
    if constexpr (R_IN_LDS) R[t] = Rl[t];
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

__global__ __launch_bounds__(1024) void frob_normalize_kernel(double* x, long long n,
                                                              double* norm_out) {
  __shared__ double part[16];
  double a = 0.0;
  for (long long i = threadIdx.x; i < n; i += 1024) a += x[i] * x[i];
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
  if (!(nrm > 0.0)) return;
  const double inv = 1.0 / nrm;
  for (long long i = threadIdx.x; i < n; i += 1024) x[i] *= inv;
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

int cholesky_inv(tn_ctx* ctx, int k, const double* G, double shift_rel, double* R, double* Rinv,
                 int* info, int batch) {
  const size_t one = (size_t)k * k * sizeof(double);
  if (one > LDS_LIMIT) TN_FAIL(ctx, TN_EINVAL, "cholesky_inv supports k <= 137 (k=%d)", k);
  if (batch < 1) return TN_OK;
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

int frob_normalize(tn_ctx* ctx, double* x, long long n, double* norm_out) {
  hipLaunchKernelGGL(frob_normalize_kernel, dim3(1), dim3(1024), 0, ctx->stream, x, n, norm_out);
  TN_HIP(ctx, hipGetLastError());
  return TN_OK;
}

int fill_random(tn_ctx* ctx, double* x, long long n, unsigned long long seed) {
  if (n <= 0) return TN_OK;
  hipLaunchKernelGGL(fill_random_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     ctx->stream, x, n, seed);
  TN_HIP(ctx, hipGetLastError());
  return TN_OK;
}
