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
constexpr int SVD_THREADS = 512;
constexpr int SVD_WAVES = SVD_THREADS / 64;

__global__ __launch_bounds__(SVD_THREADS) void jacobi_svd_kernel(
    const double* __restrict__ Ain, int lda, long long sA, double* __restrict__ U, int ldu,
    long long sU, double* __restrict__ S, long long sS, double* __restrict__ V, int ldv,
    long long sV, int m, int n, double* __restrict__ work, int max_sweeps, double tol) {
  const long long b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double* A = Ain + b * sA;
  double* X = work + b * (long long)(m * n + n * n);  // X[j*m + i]
  double* W = X + (long long)m * n;                    // W[j*n + i] (V columns)
  __shared__ double off_w[SVD_WAVES];
  __shared__ double colnorm[512];
  __shared__ int perm[512];
  __shared__ int done;

  for (long long t = tid; t < (long long)m * n; t += SVD_THREADS) {
    const int i = (int)(t / n), j = (int)(t % n);
    X[(long long)j * m + i] = A[(long long)i * lda + j];
  }
  for (long long t = tid; t < (long long)n * n; t += SVD_THREADS) {
    const int i = (int)(t / n), j = (int)(t % n);
    W[(long long)j * n + i] = (i == j) ? 1.0 : 0.0;
  }
  if (tid == 0) done = 0;
  __syncthreads();

  const int N = (n + 1) & ~1;  // players incl. a dummy when n is odd
  for (int sweep = 0; sweep < max_sweeps && n > 1; ++sweep) {
    double offmax = 0.0;
    for (int r = 0; r < N - 1; ++r) {
      for (int q = wave; q < N / 2; q += SVD_WAVES) {
        const int p0 = (q == 0) ? 0 : 1 + ((q - 1 + r) % (N - 1));
        const int p1 = 1 + ((N - 2 - q + r) % (N - 1));
        if (p0 >= n || p1 >= n) continue;
        const int p = min(p0, p1), qq = max(p0, p1);
        double* xp = X + (long long)p * m;
        double* xq = X + (long long)qq * m;
        double a = 0.0, bb = 0.0, g = 0.0;
        for (int i = lane; i < m; i += 64) {
          const double u = xp[i], v = xq[i];
          a += u * u;
          bb += v * v;
          g += u * v;
        }
        a = wave_sum(a);
        bb = wave_sum(bb);
        g = wave_sum(g);
        const double scale = sqrt(a * bb);
        if (scale == 0.0 || fabs(g) <= tol * scale) continue;
        offmax = fmax(offmax, fabs(g) / scale);
        const double z = (bb - a) / (2.0 * g);
        const double t = (z >= 0.0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int i = lane; i < m; i += 64) {
          const double u = xp[i], v = xq[i];
          xp[i] = c * u - s * v;
          xq[i] = s * u + c * v;
        }
        double* wp = W + (long long)p * n;
        double* wq = W + (long long)qq * n;
        for (int i = lane; i < n; i += 64) {
          const double u = wp[i], v = wq[i];
          wp[i] = c * u - s * v;
          wq[i] = s * u + c * v;
        }
      }
      __syncthreads();
    }
    if (lane == 0) off_w[wave] = offmax;
    __syncthreads();
    if (tid == 0) {
      double mx = 0.0;
      for (int w = 0; w < SVD_WAVES; ++w) mx = fmax(mx, off_w[w]);
      done = (mx <= tol) ? 1 : 0;
    }
    __syncthreads();
    if (done) break;
  }
  // column norms = singular values
  for (int j = wave; j < n; j += SVD_WAVES) {
    double a = 0.0;
    for (int i = lane; i < m; i += 64) a += X[(long long)j * m + i] * X[(long long)j * m + i];
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
    // argmax |x| over the column (first occurrence)
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int i = lane; i < m; i += 64) {
      const double v = fabs(X[(long long)j * m + i]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    const double sg = (bi < m && X[(long long)j * m + bi] < 0.0) ? -1.0 : 1.0;
    if (U)
      for (int i = lane; i < m; i += 64)
        U[b * sU + (long long)i * ldu + r] = sg * inv * X[(long long)j * m + i];
    if (V)
      for (int i = lane; i < n; i += 64)
        V[b * sV + (long long)i * ldv + r] = sg * W[(long long)j * n + i];
    if (S && lane == 0) S[b * sS + r] = sj;
  }
}

// ---------------------------------------------------------------------------
// Cholesky of G + shift I (right-looking, k steps) and the inverse of the
// upper factor by back substitution, one column per thread.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void cholesky_inv_kernel(const double* __restrict__ G, int k,
                                                           double shift_rel,
                                                           double* __restrict__ R,
                                                           double* __restrict__ Rinv,
                                                           double* __restrict__ Wk,
                                                           int* __restrict__ info) {
  const int tid = threadIdx.x;
  __shared__ double shift;
  __shared__ int fail;
  if (tid == 0) {
    double tr = 0.0;
    for (int i = 0; i < k; ++i) tr += G[i * k + i];
    shift = shift_rel * tr;
    fail = 0;
  }
  __syncthreads();
  for (int t = tid; t < k * k; t += 256) {
    const int i = t / k, j = t % k;
    Wk[t] = G[t] + ((i == j) ? shift : 0.0);
    R[t] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    if (tid == 0) {
      const double dj = Wk[j * k + j];
      if (!(dj > 0.0)) {
        fail = j + 1;
      } else {
        R[j * k + j] = sqrt(dj);
      }
    }
    __syncthreads();
    if (fail) break;
    const double rjj = R[j * k + j];
    for (int c = j + 1 + tid; c < k; c += 256) R[j * k + c] = Wk[j * k + c] / rjj;
    __syncthreads();
    const int w = k - j - 1;
    for (int t = tid; t < w * w; t += 256) {
      const int r = j + 1 + t / w, c = j + 1 + t % w;
      if (r <= c) Wk[r * k + c] -= R[j * k + r] * R[j * k + c];
    }
    __syncthreads();
  }
  if (tid == 0) *info = fail;
  if (fail) return;
  // Rinv column c: solve R x = e_c from the bottom
  for (int c = tid; c < k; c += 256) {
    for (int i = k - 1; i >= 0; --i) {
      if (i > c) {
        Rinv[i * k + c] = 0.0;
        continue;
      }
      double s = (i == c) ? 1.0 : 0.0;
      for (int l = i + 1; l <= c; ++l) s -= R[i * k + l] * Rinv[l * k + c];
      Rinv[i * k + c] = s / R[i * k + i];
    }
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

}  // namespace

int jacobi_svd(tn_ctx* ctx, int batch, int m, int n, double* A, int lda, long long sA, double* U,
               int ldu, long long sU, double* S, long long sS, double* V, int ldv, long long sV) {
  if (m < n) TN_FAIL(ctx, TN_EINVAL, "jacobi_svd needs m >= n (m=%d n=%d)", m, n);
  if (n > 512) TN_FAIL(ctx, TN_EINVAL, "jacobi_svd supports n <= 512 (n=%d)", n);
  if (batch <= 0 || n <= 0) return TN_OK;
  const size_t mark = ctx->arena_off;  // stream order makes the slice reusable afterwards
  double* work = ws_alloc<double>(ctx, (size_t)batch * (m * n + n * n));
  if (!work) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted in jacobi_svd");
  const double tol = 2.220446049250313e-16 * sqrt((double)m);
  hipLaunchKernelGGL(jacobi_svd_kernel, dim3(batch), dim3(SVD_THREADS), 0, ctx->stream, A, lda,
                     sA, U, ldu, sU, S, sS, V, ldv, sV, m, n, work, 80, tol);
  TN_HIP(ctx, hipGetLastError());
  ctx->arena_off = mark;
  return TN_OK;
}

int cholesky_inv(tn_ctx* ctx, int k, const double* G, double shift_rel, double* R, double* Rinv,
                 int* info) {
  const size_t mark = ctx->arena_off;
  double* wk = ws_alloc<double>(ctx, (size_t)k * k);
  if (!wk) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted in cholesky_inv");
  hipLaunchKernelGGL(cholesky_inv_kernel, dim3(1), dim3(256), 0, ctx->stream, G, k, shift_rel, R,
                     Rinv, wk, info);
  TN_HIP(ctx, hipGetLastError());
  ctx->arena_off = mark;
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
