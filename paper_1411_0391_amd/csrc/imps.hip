// 1D iMPS environment and the iTEBD step (Sec. III and V of the paper).
//
// The environment of a bond of an infinite MPS is the pair of dominant
// eigenvectors of the unit-cell transfer matrix: the Gram matrices of the
// half-infinite chains on either side of the bond.  They are found by power
// iteration in one persistent workgroup per direction, with the cell tensors,
// the iterate and the intermediate held in LDS (chi <= 36 for a two-site cell
// with d = 2; larger cells use a global scratch buffer).  The truncation
// factors the fixed points (vl = Y^T Y, vr = X X^T) with the small Jacobi
// SVD, takes the SVD of Y X and keeps chi singular pairs (Eq. (EqCanoPQ1)).
#include <cmath>
#include <mutex>
#include <cstring>

#include "bondnet.h"
#include "common.h"

namespace {

constexpr int TM_THREADS = 1024;

__device__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < TM_THREADS / 64; ++i) s += red[i];
  return s;
}

typedef double tm_dv4 __attribute__((ext_vector_type(4)));

// C = A B for small matrices given by element accessors, on FP64 MFMA
// 16x16x4 tiles: each wave of the workgroup takes 16 x 16 output tiles in
// turn; lane (hi, lo) = (lane / 16, lane % 16) supplies A[row lo][k hi] and
// B[k hi][col lo] of each k-step and holds C[row hi + 4 r][col lo].  Rows,
// columns and k past the sizes read as zero and are not written.
template <class FA, class FB, class FC>
__device__ void small_gemm(int Mr, int Nc, int Kd, FA a, FB b, FC c) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int hi = lane >> 4, lo = lane & 15;
  const int tn = (Nc + 15) / 16, nt = ((Mr + 15) / 16) * tn, nk = (Kd + 3) / 4;
  for (int tile = wv; tile < nt; tile += nw) {
    const int r0 = (tile / tn) * 16, c0 = (tile % tn) * 16;
    const int ra = r0 + lo, cb = c0 + lo;
    tm_dv4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int q = 0; q < nk; ++q) {
      const int k = 4 * q + hi;
      const double av = (ra < Mr && k < Kd) ? a(ra, k) : 0.0;
      const double bv = (k < Kd && cb < Nc) ? b(k, cb) : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = r0 + hi + 4 * r;
      if (row < Mr && cb < Nc) c(row, cb, acc[r]);
    }
  }
}

// v <- one application of the cell transfer matrix (left: v -> sum K^T v B
// site by site in cell order; right: v -> sum K v B^T, last site first),
// each site as two small products on MFMA
__device__ void tm_apply(const double* K, const double* B, int nsite, int chi, int d, int left,
                         double* v, double* x) {
  const int cdc = chi * d * chi, dn = d * chi;
  for (int q = 0; q < nsite; ++q) {
    const int site = left ? q : nsite - 1 - q;
    const double* k = K + (long long)site * cdc;
    const double* bb = B + (long long)site * cdc;
    if (left) {
      // x[b][(s c)] = sum_a v[a][b] k[a][(s c)]
      small_gemm(chi, dn, chi, [&](int r, int kk) { return v[kk * chi + r]; },
                 [&](int kk, int c) { return k[kk * dn + c]; },
                 [&](int r, int c, double val) { x[r * dn + c] = val; });
      __syncthreads();
      // v[c][e] = sum_{(b s)} x[(b s)][c] bb[(b s)][e]
      small_gemm(chi, chi, dn, [&](int r, int kk) { return x[kk * chi + r]; },
                 [&](int kk, int c) { return bb[kk * chi + c]; },
                 [&](int r, int c, double val) { v[r * chi + c] = val; });
    } else {
      // x[(a s)][e] = sum_c k[(a s)][c] v[c][e]
      small_gemm(dn, chi, chi, [&](int r, int kk) { return k[r * chi + kk]; },
                 [&](int kk, int c) { return v[kk * chi + c]; },
                 [&](int r, int c, double val) { x[r * chi + c] = val; });
      __syncthreads();
      // v[a][b] = sum_{(s e)} x[a][(s e)] bb[b][(s e)]
      small_gemm(chi, chi, dn, [&](int r, int kk) { return x[r * dn + kk]; },
                 [&](int kk, int c) { return bb[c * dn + kk]; },
                 [&](int r, int c, double val) { v[r * chi + c] = val; });
    }
    __syncthreads();
  }
}

// Power iteration: block 0 left, block 1 right.  The iterate is kept at unit
// Frobenius norm with positive trace; stops when it moves by less than tol.
// GLOBAL: the working set lives in gwork instead of LDS (a compile-time
// choice, so that LDS accesses compile to LDS instructions)
template <bool GLOBAL>
__global__ __launch_bounds__(TM_THREADS) void tm_power_kernel(
    const double* __restrict__ kets, const double* __restrict__ bras, int nsite, int chi, int d,
    double* __restrict__ vout, double* __restrict__ eta, int* __restrict__ iters, double tol,
    int max_iter, int warm, double* __restrict__ gwork) {
  extern __shared__ double lds[];
  __shared__ double red[TM_THREADS / 64];
  // blocks 2p and 2p + 1: the left and right fixed points of problem p
  const int left = (blockIdx.x & 1) == 0 ? 1 : 0;
  kets += (long long)(blockIdx.x >> 1) * nsite * chi * d * chi;
  bras += (long long)(blockIdx.x >> 1) * nsite * chi * d * chi;
  const int tid = threadIdx.x;
  const int cdc = chi * d * chi, cc = chi * chi;
  const long long per = 2LL * nsite * cdc + 2LL * cc + cdc;
  double* base;
  if constexpr (GLOBAL)
    base = gwork + blockIdx.x * per;
  else
    base = lds;
  double* K = base;
  double* B = K + (long long)nsite * cdc;
  double* v = B + (long long)nsite * cdc;
  double* w = v + cc;
  double* x = w + cc;
  for (long long t = tid; t < (long long)nsite * cdc; t += TM_THREADS) {
    K[t] = kets[t];
    B[t] = bras[t];
  }
  double* vo = vout + blockIdx.x * cc;
  for (int t = tid; t < cc; t += TM_THREADS)
    v[t] = warm ? vo[t] : ((t / chi == t % chi) ? 1.0 : 0.0);
  __syncthreads();
  // normalise the start
  {
    double a = 0.0;
    for (int t = tid; t < cc; t += TM_THREADS) a += v[t] * v[t];
    const double nrm = sqrt(block_sum(a, red));
    double tr = 0.0;
    for (int i = tid; i < chi; i += TM_THREADS) tr += v[i * chi + i];
    tr = block_sum(tr, red);
    const double f = (tr < 0.0 ? -1.0 : 1.0) / (nrm > 0.0 ? nrm : 1.0);
    for (int t = tid; t < cc; t += TM_THREADS) v[t] *= f;
    __syncthreads();
  }
  int it = 0;
  double ev = 0.0;
  for (it = 1; it <= max_iter; ++it) {
    for (int t = tid; t < cc; t += TM_THREADS) w[t] = v[t];
    __syncthreads();
    tm_apply(K, B, nsite, chi, d, left, w, x);
    double a = 0.0, ip = 0.0, tr = 0.0;
    for (int t = tid; t < cc; t += TM_THREADS) {
      a += w[t] * w[t];
      ip += w[t] * v[t];
    }
    for (int i = tid; i < chi; i += TM_THREADS) tr += w[i * chi + i];
    const double nrm = sqrt(block_sum(a, red));
    ev = block_sum(ip, red);
    tr = block_sum(tr, red);
    const double f = (tr < 0.0 ? -1.0 : 1.0) / (nrm > 0.0 ? nrm : 1.0);
    double dd = 0.0;
    for (int t = tid; t < cc; t += TM_THREADS) {
      const double nv = w[t] * f;
      dd += (nv - v[t]) * (nv - v[t]);
      v[t] = nv;
    }
    const double diff = sqrt(block_sum(dd, red));
    if (!(diff >= tol)) break;  // also stops on NaN
  }
  for (int t = tid; t < cc; t += TM_THREADS) vo[t] = v[t];
  if (tid == 0) {
    eta[blockIdx.x] = ev;
    iters[blockIdx.x] = it;
  }
}

// Restarted Arnoldi for the same fixed point: per restart an m-step Krylov
// basis V_0 = v, V_{j+1} ~ (TM - h) V_j, orthogonalised by two passes of
// classical Gram-Schmidt, the Hessenberg matrix H of TM on the basis, and
// the dominant Ritz pair (theta, y) of H by repeated squaring of H applied
// to e_0 (normalised); v <- V y with unit norm and positive trace.  The
// Arnoldi relation gives the residual |TM v - theta v| = |H[m][m-1] y[m-1]|;
// the restarts end when it is below tol |theta|.  Near the critical field,
// where the transfer matrix's gap is small, this takes an order of magnitude
// fewer applications than the power iteration.  kry: (TM_KRYLOV + 1) chi^2
// doubles per side.  iters counts applications (>= max_iter when not
// converged).
constexpr int TM_KRYLOV = 12;

// Orders the LDS accesses of one wave among themselves (a wave's LDS
// instructions complete in order; this keeps the compiler from moving them
// across the point).  Only for code that a single wave runs: a workgroup
// barrier there would pair with the other waves' barriers.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <bool GLOBAL>
__global__ __launch_bounds__(TM_THREADS) void tm_krylov_kernel(
    const double* __restrict__ kets, const double* __restrict__ bras, int nsite, int chi, int d,
    double* __restrict__ vout, double* __restrict__ eta, int* __restrict__ iters, double tol,
    int max_iter, int warm, double* __restrict__ gwork, double* __restrict__ kry) {
  constexpr int M = TM_KRYLOV;
  constexpr int NW = TM_THREADS / 64;
  extern __shared__ double lds[];
  __shared__ double red[NW];
  __shared__ double part[NW][M];
  __shared__ double H[(M + 1) * M];
  __shared__ double Hp[M * M], Hq[M * M];
  __shared__ double hcol[M + 1], y[M], sc[4];
  // blocks 2p and 2p + 1: the left and right fixed points of problem p
  const int left = (blockIdx.x & 1) == 0 ? 1 : 0;
  kets += (long long)(blockIdx.x >> 1) * nsite * chi * d * chi;
  bras += (long long)(blockIdx.x >> 1) * nsite * chi * d * chi;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int cdc = chi * d * chi, cc = chi * chi;
  const long long per = 2LL * nsite * cdc + 2LL * cc + cdc;
  double* base;
  if constexpr (GLOBAL)
    base = gwork + blockIdx.x * per;
  else
    base = lds;
  double* K = base;
  double* B = K + (long long)nsite * cdc;
  double* v = B + (long long)nsite * cdc;
  double* w = v + cc;
  double* x = w + cc;
  double* V = kry + (long long)blockIdx.x * (M + 1) * cc;
  for (long long t = tid; t < (long long)nsite * cdc; t += TM_THREADS) {
    K[t] = kets[t];
    B[t] = bras[t];
  }
  double* vo = vout + blockIdx.x * cc;
  for (int t = tid; t < cc; t += TM_THREADS)
    v[t] = warm ? vo[t] : ((t / chi == t % chi) ? 1.0 : 0.0);
  __syncthreads();
  int mv = 0;
  double theta = 0.0, res_prev = INFINITY;
  bool conv = false;
  while (!conv && mv < max_iter) {
    // V_0 = v / |v|
    {
      double a = 0.0;
      for (int t = tid; t < cc; t += TM_THREADS) a += v[t] * v[t];
      const double nrm = sqrt(block_sum(a, red));
      const double f = nrm > 0.0 ? 1.0 / nrm : 1.0;
      for (int t = tid; t < cc; t += TM_THREADS) V[t] = v[t] * f;
    }
    __syncthreads();
    int m = 0;
    for (int j = 0; j < M; ++j) {
      for (int t = tid; t < cc; t += TM_THREADS) w[t] = V[(long long)j * cc + t];
      __syncthreads();
      tm_apply(K, B, nsite, chi, d, left, w, x);
      ++mv;
      if (tid <= j) hcol[tid] = 0.0;
      // two passes of classical Gram-Schmidt against V_0..V_j
      for (int pass = 0; pass < 2; ++pass) {
        double hp[M];
#pragma unroll
        for (int i = 0; i < M; ++i) hp[i] = 0.0;
        for (int t = tid; t < cc; t += TM_THREADS) {
          const double wt = w[t];
#pragma unroll
          for (int i = 0; i < M; ++i)
            if (i <= j) hp[i] += V[(long long)i * cc + t] * wt;
        }
#pragma unroll
        for (int i = 0; i < M; ++i) {
          if (i <= j) {  // uniform over the wave
            double a = hp[i];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
            if (lane == 0) part[wv][i] = a;
          }
        }
        __syncthreads();
        if (tid <= j) {
          double a = 0.0;
          for (int q = 0; q < NW; ++q) a += part[q][tid];
          hcol[tid] += a;
          y[tid] = a;  // this pass's coefficients
        }
        __syncthreads();
        for (int t = tid; t < cc; t += TM_THREADS) {
          double a = w[t];
          for (int i = 0; i <= j; ++i) a -= y[i] * V[(long long)i * cc + t];
          w[t] = a;
        }
        __syncthreads();
      }
      double a = 0.0;
      for (int t = tid; t < cc; t += TM_THREADS) a += w[t] * w[t];
      const double hn = sqrt(block_sum(a, red));
      if (tid <= j) H[tid * M + j] = hcol[tid];
      if (tid == 0) H[(j + 1) * M + j] = hn;
      for (int i = j + 2 + tid; i <= M; i += TM_THREADS) H[i * M + j] = 0.0;
      m = j + 1;
      // an invariant subspace (or a zero map): the Ritz pair is exact
      const bool breakdown = !(hn > 1e-14 * fabs(hcol[0]) + 1e-300);
      if (breakdown || j == M - 1) {
        __syncthreads();
        break;
      }
      const double f = 1.0 / hn;
      for (int t = tid; t < cc; t += TM_THREADS) V[(long long)(j + 1) * cc + t] = w[t] * f;
      __syncthreads();
    }
    // dominant Ritz pair of the m x m leading block of H (wave 0): y is the
    // normalised first column of H^(2^k), squaring until it stops changing
    if (wv == 0) {
      for (int e = lane; e < M * M; e += 64) {
        const int r = e / M, c = e % M;
        Hp[e] = (r < m && c < m) ? H[r * M + c] : 0.0;
      }
      wave_sync();
      double yprev[M];
      for (int q = 0; q < M; ++q) yprev[q] = q == 0 ? 1.0 : 0.0;
      for (int sq = 0; sq < 60; ++sq) {
        // Hq = Hp Hp, scaled to unit max norm
        for (int e = lane; e < M * M; e += 64) {
          const int r = e / M, c = e % M;
          double acc = 0.0;
          for (int q = 0; q < M; ++q) acc += Hp[r * M + q] * Hp[q * M + c];
          Hq[e] = acc;
        }
        wave_sync();
        double mx = 0.0;
        for (int e = lane; e < M * M; e += 64) mx = fmax(mx, fabs(Hq[e]));
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
        const double f = mx > 0.0 ? 1.0 / mx : 1.0;
        for (int e = lane; e < M * M; e += 64) Hp[e] = Hq[e] * f;
        wave_sync();
        // candidate y: the first column, unit norm, positive first nonzero
        double nrm = 0.0;
        for (int q = 0; q < m; ++q) nrm += Hp[q * M] * Hp[q * M];
        nrm = sqrt(nrm);
        double sgn = 1.0;
        for (int q = 0; q < m; ++q)
          if (fabs(Hp[q * M]) > 1e-8 * nrm) {
            sgn = Hp[q * M] < 0.0 ? -1.0 : 1.0;
            break;
          }
        double dmax = 0.0;
        for (int q = 0; q < M; ++q) {
          const double yq = (q < m && nrm > 0.0) ? sgn * Hp[q * M] / nrm : 0.0;
          dmax = fmax(dmax, fabs(yq - yprev[q]));
          yprev[q] = yq;
        }
        if (dmax < 1e-15) break;
      }
      if (lane < M) y[lane] = yprev[lane];
      wave_sync();
      if (lane == 0) {
        // theta from the Rayleigh quotient of H on y; residual from the
        // Arnoldi relation
        double num = 0.0, den = 0.0;
        for (int r = 0; r < m; ++r) {
          double hy = 0.0;
          for (int c = 0; c < m; ++c) hy += H[r * M + c] * y[c];
          num += y[r] * hy;
          den += y[r] * y[r];
        }
        sc[1] = den > 0.0 ? num / den : 0.0;
        sc[2] = fabs(H[m * M + (m - 1)] * y[m - 1]);
      }
    }
    __syncthreads();
    theta = sc[1];
    const double res = sc[2];
    // v = V y, unit norm and positive trace
    for (int t = tid; t < cc; t += TM_THREADS) {
      double a = 0.0;
      for (int i = 0; i < m; ++i) a += y[i] * V[(long long)i * cc + t];
      v[t] = a;
    }
    __syncthreads();
    {
      double a = 0.0, tr = 0.0;
      for (int t = tid; t < cc; t += TM_THREADS) a += v[t] * v[t];
      for (int i = tid; i < chi; i += TM_THREADS) tr += v[i * chi + i];
      const double nrm = sqrt(block_sum(a, red));
      tr = block_sum(tr, red);
      const double f = (tr < 0.0 ? -1.0 : 1.0) / (nrm > 0.0 ? nrm : 1.0);
      for (int t = tid; t < cc; t += TM_THREADS) v[t] *= f;
      __syncthreads();
    }
    // converged, or within 100x of the target with the residual no longer
    // halving per restart (its rounding floor); both false on NaN
    conv = res <= tol * fabs(theta) || (res <= 100.0 * tol * fabs(theta) && res > 0.5 * res_prev);
    res_prev = res;
  }
  for (int t = tid; t < cc; t += TM_THREADS) vo[t] = v[t];
  if (tid == 0) {
    eta[blockIdx.x] = theta;
    iters[blockIdx.x] = conv ? mv : (mv > max_iter ? mv : max_iter);
  }
}

// vr <- vr / sum(vl * vr)
__global__ void pair_normalize_kernel(const double* __restrict__ vl, double* __restrict__ vr,
                                      int cc) {
  __shared__ double red[4];
  double a = 0.0;
  for (int t = threadIdx.x; t < cc; t += 256) a += vl[t] * vr[t];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  const double s = red[0] + red[1] + red[2] + red[3];
  const double inv = s != 0.0 ? 1.0 / s : 0.0;
  for (int t = threadIdx.x; t < cc; t += 256) vr[t] *= inv;
}

// Theta[(i,a)][s][(j,b)] = sum_t g[a][b][s][t] A[i][t][j]
__global__ void impo_apply_kernel(const double* __restrict__ g, const double* __restrict__ A,
                                  double* __restrict__ Th, int chi, int d, int kap) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)chi * kap * d * chi * kap;
  if (t >= tot) return;
  long long r = t;
  const int b = r % kap; r /= kap;
  const int j = r % chi; r /= chi;
  const int s = r % d; r /= d;
  const int a = r % kap; r /= kap;
  const int i = (int)r;
  double acc = 0.0;
  for (int tt = 0; tt < d; ++tt)
    acc += g[((a * kap + b) * d + s) * d + tt] * A[((long long)i * d + tt) * chi + j];
  Th[t] = acc;
}

// Square-root factors of a symmetric positive semi-definite v = W S W^T
// given its SVD (U = W, S): F = W sqrt(S) and Finv = (W / sqrt(S))^T,
// dropping S < 1e-14 S_max (F, Finv n x n).
__global__ void sqrt_factors_kernel(const double* __restrict__ U, const double* __restrict__ S,
                                    int n, double* __restrict__ F, double* __restrict__ Finv) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n) return;
  const int i = t / n, j = t % n;
  const double sj = S[j];
  const bool keep = sj > 1e-14 * S[0];
  const double sq = keep ? sqrt(sj) : 0.0;
  F[i * n + j] = U[i * n + j] * sq;
  Finv[j * n + i] = keep ? U[i * n + j] / sq : 0.0;
}

// P = Yinv[:, :] U[:, :chi] sqrt(S) with Yinv = W / sqrt(s) (columns),
// computed by the host as a product; here: scale the chi kept columns of a
// matrix by sqrt(S) (cols) or its rows (rows = 1).
__global__ void scale_sqrt_kernel(double* __restrict__ X, int rows, int cols, int ld,
                                  const double* __restrict__ S, int by_rows) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * cols) return;
  const int i = t / cols, j = t % cols;
  X[i * ld + j] *= sqrt(fmax(S[by_rows ? i : j], 0.0));
}

// kept spectrum (normalised) and discarded weight of one bond
__global__ void spectrum_kernel(const double* __restrict__ S, int n, int chi,
                                double* __restrict__ lam, double* __restrict__ err) {
  if (threadIdx.x != 0) return;
  double kept = 0.0, tot = 0.0;
  for (int i = 0; i < n; ++i) {
    tot += S[i] * S[i];
    if (i < chi) kept += S[i] * S[i];
  }
  const double inv = kept > 0.0 ? 1.0 / sqrt(kept) : 0.0;
  for (int i = 0; i < chi; ++i) lam[i] = (i < n) ? S[i] * inv : 0.0;
  *err += tot > 0.0 ? (tot - kept) / tot : 0.0;
}

// TFIM energy per site from the two bond RDMs (4x4, (s1 s2),(s1' s2'))
__global__ void tfim1d_energy_kernel(const double* __restrict__ r0, const double* __restrict__ r1,
                                     double J, double h, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  const double zz[4] = {1.0, -1.0, -1.0, 1.0};
  double tr0 = 0.0, tr1 = 0.0, z0 = 0.0, z1 = 0.0;
  for (int i = 0; i < 4; ++i) {
    tr0 += r0[i * 4 + i];
    tr1 += r1[i * 4 + i];
    z0 += zz[i] * r0[i * 4 + i];
    z1 += zz[i] * r1[i * 4 + i];
  }
  // <sx (x) 1> and <1 (x) sx> on the first bond: index (s1 s2) = 2 s1 + s2
  double x1 = 0.0, x2 = 0.0;
  for (int s2 = 0; s2 < 2; ++s2) {
    x1 += r0[(0 * 2 + s2) * 4 + (1 * 2 + s2)] + r0[(1 * 2 + s2) * 4 + (0 * 2 + s2)];
  }
  for (int s1 = 0; s1 < 2; ++s1) {
    x2 += r0[(s1 * 2 + 0) * 4 + (s1 * 2 + 1)] + r0[(s1 * 2 + 1) * 4 + (s1 * 2 + 0)];
  }
  *out = -J * 0.5 * (z0 / tr0 + z1 / tr1) - h * 0.5 * (x1 + x2) / tr0;
}

// Doubles of the power kernel's working set per side (two cell tensors, two
// iterates and one intermediate), and whether it exceeds LDS.
size_t tm_work_per_side(int nsite, int chi, int d) {
  return 2ULL * nsite * chi * d * chi + 2ULL * chi * chi + (size_t)chi * d * chi;
}
bool tm_work_in_global(int nsite, int chi, int d) {
  return tm_work_per_side(nsite, chi, d) * sizeof(double) > 150 * 1024;
}

// Both fixed points: gwork holds 2 tm_work_per_side doubles when the working
// set exceeds LDS (null: taken from the arena).
// nprob independent problems in one launch: problem p's cell at
// kets/bras + p nsite chi d chi, its fixed points at v2 + 2 p chi^2, its
// eta and iteration counts at index 2 p (left) and 2 p + 1 (right).
int tm_pair(tn_ctx* ctx, int nsite, int chi, int d, const double* kets, const double* bras,
            double* v2 /*[nprob][2][chi][chi]*/, double* eta_d, int* it_d, double tol,
            int max_iter, int warm, double* gwork = nullptr, bool krylov = false,
            int nprob = 1) {
  const size_t per = tm_work_per_side(nsite, chi, d);
  const unsigned blocks = 2u * (unsigned)nprob;
  size_t dyn = per * sizeof(double);
  if (!tm_work_in_global(nsite, chi, d)) {
    gwork = nullptr;
  } else {
    // a caller's gwork holds the two sides of one problem
    if (gwork && nprob != 1) TN_FAIL(ctx, TN_EINVAL, "caller workspace for one problem only");
    if (!gwork) gwork = ws_alloc<double>(ctx, blocks * per);
    if (!gwork) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted (transfer matrix)");
    dyn = 0;
  }
  if (krylov) {
    double* kry = ws_alloc<double>(ctx, blocks * (size_t)(TM_KRYLOV + 1) * chi * chi);
    if (!kry) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted (Krylov basis)");
    if (gwork)
      hipLaunchKernelGGL(tm_krylov_kernel<true>, dim3(blocks), dim3(TM_THREADS), dyn,
                         ctx->stream, kets, bras, nsite, chi, d, v2, eta_d, it_d, tol, max_iter,
                         warm, gwork, kry);
    else
      hipLaunchKernelGGL(tm_krylov_kernel<false>, dim3(blocks), dim3(TM_THREADS), dyn,
                         ctx->stream, kets, bras, nsite, chi, d, v2, eta_d, it_d, tol, max_iter,
                         warm, gwork, kry);
  } else if (gwork)
    hipLaunchKernelGGL(tm_power_kernel<true>, dim3(blocks), dim3(TM_THREADS), dyn, ctx->stream,
                       kets, bras, nsite, chi, d, v2, eta_d, it_d, tol, max_iter, warm, gwork);
  else
    hipLaunchKernelGGL(tm_power_kernel<false>, dim3(blocks), dim3(TM_THREADS), dyn, ctx->stream,
                       kets, bras, nsite, chi, d, v2, eta_d, it_d, tol, max_iter, warm, gwork);
  TN_HIP(ctx, hipGetLastError());
  const size_t cc = (size_t)chi * chi;
  for (int p = 0; p < nprob; ++p)
    hipLaunchKernelGGL(pair_normalize_kernel, dim3(1), dim3(256), 0, ctx->stream, v2 + 2 * p * cc,
                       v2 + (2 * p + 1) * cc, chi * chi);
  TN_HIP(ctx, hipGetLastError());
  return TN_OK;
}

// Host-side iMPO g[a][b][s][t] of the TFIM (Eq. (iMPO1)): g = gF R_a L_b gF,
// gF = exp(dt h sx / 2), exp(dt J sz sz) = sum_k L_k (x) R_k with
// L = {sqrt(cosh) 1, sqrt|sinh| sz}, R = {sqrt(cosh) 1, sign(sinh) sqrt|sinh| sz}.
void tfim_impo(double J, double h, double dt, double g[2][2][2][2]) {
  const double c = cosh(0.5 * dt * h), s = sinh(0.5 * dt * h);
  const double gf[2][2] = {{c, s}, {s, c}};
  const double ch = cosh(dt * J), sh = sinh(dt * J);
  const double l[2] = {sqrt(ch), sqrt(fabs(sh))};
  const double r[2] = {sqrt(ch), (sh < 0 ? -1.0 : 1.0) * sqrt(fabs(sh))};
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      // diagonal middle factor: R_a L_b, sz powers add
      double mid[2];
      for (int q = 0; q < 2; ++q) {
        const double za = (a == 1) ? (q == 0 ? 1.0 : -1.0) : 1.0;
        const double zb = (b == 1) ? (q == 0 ? 1.0 : -1.0) : 1.0;
        mid[q] = r[a] * za * l[b] * zb;
      }
      for (int s1 = 0; s1 < 2; ++s1)
        for (int t1 = 0; t1 < 2; ++t1) {
          double acc = 0.0;
          for (int q = 0; q < 2; ++q) acc += gf[s1][q] * mid[q] * gf[q][t1];
          g[a][b][s1][t1] = acc;
        }
    }
}

}  // namespace

// Workspace layout of env1d (doubles): [0, 4 n^2) warm fixed points
// (bond 0: vl, vr; bond 1: vl, vr) with n = kappa chi; then the recycling
// factors Lf[2][chi][n] and Rf[2][n][chi]; then 16 flags/scalars.
size_t env1d_doubles(int chi, int d) {
  (void)d;
  const size_t n = 2 * (size_t)chi;
  return 4 * n * n + 4 * (size_t)chi * n + 16;
}

// Copy the fixed points out and read the eigenvalue and iteration counts
// back through the context's pinned buffer.
static int tm_finish(tn_ctx* ctx, int chi, const double* v2, const double* ed, const int* itd,
              double* vl, double* vr, double* eta, int* iters, int max_iter) {
  const size_t cc = (size_t)chi * chi;
  TN_HIP(ctx, hipMemcpyAsync(vl, v2, cc * 8, hipMemcpyDeviceToDevice, ctx->stream));
  TN_HIP(ctx, hipMemcpyAsync(vr, v2 + cc, cc * 8, hipMemcpyDeviceToDevice, ctx->stream));
  double* he = ctx->host_scratch;
  int* hi = reinterpret_cast<int*>(ctx->host_scratch + 2);
  TN_HIP(ctx, hipMemcpyAsync(he, ed, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  TN_HIP(ctx, hipMemcpyAsync(hi, itd, 2 * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (eta) *eta = he[0];
  if (iters) *iters = hi[0] > hi[1] ? hi[0] : hi[1];
  if (!std::isfinite(he[0]) || !std::isfinite(he[1]))
    TN_FAIL(ctx, TN_ENUMERIC, "non-finite transfer-matrix eigenvalue");
  return (hi[0] >= max_iter || hi[1] >= max_iter) ? TN_NOT_CONVERGED : TN_OK;
}

int tm_fixed_point_impl(tn_ctx* ctx, int n_sites, int chi, int d, const double* ket,
                        const double* bra, double* vl, double* vr, double* eta, double tol,
                        int max_iter, int* iters, int flags) {
  if (n_sites < 1 || chi < 1 || d < 1 || !ket || !bra || !vl || !vr || max_iter < 1)
    TN_FAIL(ctx, TN_EINVAL, "bad tm_fixed_point arguments");
  TN_TRY(ws_reserve(ctx, 2 * (2ULL * n_sites * chi * d * chi + 3ULL * chi * chi + chi * d * chi) *
                             8 + (4 << 20)));
  ws_reset(ctx);
  double* v2 = ws_alloc<double>(ctx, 2 * (size_t)chi * chi);
  double* ed = ws_alloc<double>(ctx, 2);
  int* itd = ws_alloc<int>(ctx, 2);
  if (!itd) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted");
  const size_t cc = (size_t)chi * chi;
  if (flags & 1) {
    TN_HIP(ctx, hipMemcpyAsync(v2, vl, cc * 8, hipMemcpyDeviceToDevice, ctx->stream));
    TN_HIP(ctx, hipMemcpyAsync(v2 + cc, vr, cc * 8, hipMemcpyDeviceToDevice, ctx->stream));
  }
  TN_TRY(tm_pair(ctx, n_sites, chi, d, ket, bra, v2, ed, itd, tol, max_iter, flags & 1));
  return tm_finish(ctx, chi, v2, ed, itd, vl, vr, eta, iters, max_iter);
}

// ---------------------------------------------------------------------------
// tm_fixed_point without allocation: the same kernels on a fixed scratch
// array.  Each GPU holds its own copy of `scratch` at its own address, taken
// once per device at context creation (the name is a host-side stand-in and
// is never passed to a kernel).
// ---------------------------------------------------------------------------

namespace {
constexpr size_t TM_NOALLOC_DOUBLES = size_t(1) << 19;  // 4 MiB
__device__ __align__(256) double scratch[TM_NOALLOC_DOUBLES];
constexpr int MAX_DEVICES = 64;
double* scratch_addr[MAX_DEVICES] = {nullptr};
std::mutex scratch_mu;
}  // namespace

int noalloc_scratch_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) return TN_EINVAL;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (scratch_addr[device]) return TN_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return TN_EHIP;
  }
  scratch_addr[device] = static_cast<double*>(p);
  return TN_OK;
}

int tm_fixed_point_noalloc_impl(tn_ctx* ctx, int n_sites, int chi, int d, const double* ket,
                                const double* bra, double* vl, double* vr, double* eta,
                                double tol, int max_iter, int* iters, int flags) {
  if (n_sites < 1 || chi < 1 || d < 1 || !ket || !bra || !vl || !vr || max_iter < 1)
    TN_FAIL(ctx, TN_EINVAL, "bad tm_fixed_point_noalloc arguments");
  double* base = (ctx->device >= 0 && ctx->device < MAX_DEVICES) ? scratch_addr[ctx->device]
                                                                 : nullptr;
  if (!base) TN_FAIL(ctx, TN_EHIP, "no scratch address for device %d", ctx->device);
  const size_t cc = (size_t)chi * chi;
  // iterate pair, eigenvalues, iteration counts, then the working set
  const size_t head = (2 * cc + 4 + 31) & ~size_t(31);
  const size_t work = tm_work_in_global(n_sites, chi, d) ? 2 * tm_work_per_side(n_sites, chi, d)
                                                         : 0;
  if (head + work > TM_NOALLOC_DOUBLES)
    TN_FAIL(ctx, TN_EINVAL,
            "chi = %d, %d sites need %zu doubles of scratch, more than the fixed %zu", chi,
            n_sites, head + work, TM_NOALLOC_DOUBLES);
  double* v2 = base;
  double* ed = base + 2 * cc;
  int* itd = reinterpret_cast<int*>(base + 2 * cc + 2);
  double* gwork = work ? base + head : nullptr;
  if (flags & 1) {
    TN_HIP(ctx, hipMemcpyAsync(v2, vl, cc * 8, hipMemcpyDeviceToDevice, ctx->stream));
    TN_HIP(ctx, hipMemcpyAsync(v2 + cc, vr, cc * 8, hipMemcpyDeviceToDevice, ctx->stream));
  }
  TN_TRY(tm_pair(ctx, n_sites, chi, d, ket, bra, v2, ed, itd, tol, max_iter, flags & 1, gwork));
  return tm_finish(ctx, chi, v2, ed, itd, vl, vr, eta, iters, max_iter);
}

namespace {

// Truncation of both bonds of the two-site Theta chain (bond 0 after site
// 0), the two bonds batched in every launch: fixed points of the cell
// ending with the left site of the bond, factors, SVD of Y X, P (n x chi)
// and Q (chi x n) per bond.
int bond_truncations(tn_ctx* ctx, int n, int chi, int d, const double* th /*[2][n][d][n]*/,
                     double* vwarm /*[2 bonds][2][n][n] in/out*/, int warm, double tol,
                     double* P /*[2][n][chi]*/, double* Q /*[2][chi][n]*/, double* lam /*[2][chi]*/,
                     double* err, int* tm_iters) {
  const size_t nn = (size_t)n * n, ndn = (size_t)n * d * n;
  double* cell = ws_alloc<double>(ctx, 4 * ndn);
  double* ed = ws_alloc<double>(ctx, 4);
  int* itd = ws_alloc<int>(ctx, 4);
  double* U = ws_alloc<double>(ctx, 4 * nn);
  double* S = ws_alloc<double>(ctx, 4 * (size_t)n);
  double* Yt = ws_alloc<double>(ctx, 2 * nn);
  double* Ytinv = ws_alloc<double>(ctx, 2 * nn);
  double* X = ws_alloc<double>(ctx, 2 * nn);
  double* Xinv = ws_alloc<double>(ctx, 2 * nn);
  double* M = ws_alloc<double>(ctx, 2 * nn);
  double* Um = ws_alloc<double>(ctx, 2 * nn);
  double* Vm = ws_alloc<double>(ctx, 2 * nn);
  double* Sm = ws_alloc<double>(ctx, 2 * (size_t)n);
  if (!Sm) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted (truncation)");
  // cell of bond b = [other site, site b]: its left fixed point ends with
  // site b, its right one starts with the other site
  for (int b = 0; b < 2; ++b) {
    TN_HIP(ctx, hipMemcpyAsync(cell + 2 * b * ndn, th + (1 - b) * ndn, ndn * 8,
                               hipMemcpyDeviceToDevice, ctx->stream));
    TN_HIP(ctx, hipMemcpyAsync(cell + (2 * b + 1) * ndn, th + b * ndn, ndn * 8,
                               hipMemcpyDeviceToDevice, ctx->stream));
  }
  TN_TRY(tm_pair(ctx, 2, n, d, cell, cell, vwarm, ed, itd, tol, 100000, warm, nullptr, true, 2));
  int hi[4];
  TN_HIP(ctx, hipMemcpyAsync(hi, itd, 4 * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  // per bond vl = Yt Yt^T (Y = Yt^T), vr = X X^T: the four SVDs at once
  TN_TRY(jacobi_svd(ctx, 4, n, n, vwarm, n, (long long)nn, U, n, (long long)nn, S, n, nullptr, 0,
                    0));
  for (int b = 0; b < 2; ++b) {
    hipLaunchKernelGGL(sqrt_factors_kernel, dim3((n * n + 255) / 256), dim3(256), 0, ctx->stream,
                       U + 2 * b * nn, S + 2 * b * n, n, Yt + b * nn, Ytinv + b * nn);
    hipLaunchKernelGGL(sqrt_factors_kernel, dim3((n * n + 255) / 256), dim3(256), 0, ctx->stream,
                       U + (2 * b + 1) * nn, S + (2 * b + 1) * n, n, X + b * nn, Xinv + b * nn);
  }
  TN_HIP(ctx, hipGetLastError());
  // M = Y X = Yt^T X ; SVD M = Um Sm Vm^T (sign-fixed)
  TN_TRY(gemm(ctx, n, n, n, Yt, n, true, X, n, false, M, n, 1.0, 0.0, 2, (long long)nn,
              (long long)nn, (long long)nn));
  TN_TRY(jacobi_svd(ctx, 2, n, n, M, n, (long long)nn, Um, n, (long long)nn, Sm, n, Vm, n,
                    (long long)nn));
  // P = Y^+ Um[:, :chi] sqrt(S) with Y^+ = Ytinv^T ; Q = sqrt(S) Vm[:, :chi]^T X^+
  TN_TRY(gemm(ctx, n, chi, n, Ytinv, n, true, Um, n, false, P, chi, 1.0, 0.0, 2, (long long)nn,
              (long long)nn, (long long)n * chi));
  TN_TRY(gemm(ctx, chi, n, n, Vm, n, true, Xinv, n, false, Q, n, 1.0, 0.0, 2, (long long)nn,
              (long long)nn, (long long)chi * n));
  for (int b = 0; b < 2; ++b) {
    hipLaunchKernelGGL(scale_sqrt_kernel, dim3((n * chi + 255) / 256), dim3(256), 0, ctx->stream,
                       P + b * n * chi, n, chi, chi, Sm + b * n, 0);
    hipLaunchKernelGGL(scale_sqrt_kernel, dim3((n * chi + 255) / 256), dim3(256), 0, ctx->stream,
                       Q + b * chi * n, chi, n, n, Sm + b * n, 1);
    hipLaunchKernelGGL(spectrum_kernel, dim3(1), dim3(1), 0, ctx->stream, Sm + b * n, n, chi,
                       lam + b * chi, err);
  }
  TN_HIP(ctx, hipGetLastError());
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *tm_iters = std::max(std::max(hi[0], hi[1]), std::max(hi[2], hi[3]));
  return TN_OK;
}

// Canonical form of a two-site A-form cell (Sec. III A) from the exact
// environments of its bonds.  With the transfer-matrix fixed points
// V_L = Y^T Y and V_R = X X^T of a bond and the SVD Y X = U S V^T, the gauge
// P = Y^+ U S^1/2 on the left site's right leg and Q = S^1/2 V^T X^+ on the
// right site's left leg leaves both environments of the bond equal to S:
// the fixed point that the paper's local iteration converges to, reached in
// one step (the iteration converges at the rate of the transfer matrix's
// gap, thousands of steps near the critical field).  Outputs: Pc, Qc
// [2][chi][chi] in the canonical sign and scale, lam_out [2][chi] (unit
// norm; may be null), Aout [2][chi][d][chi] = Qc A Pc per site, unit norm.
int canonical_1d(tn_ctx* ctx, const BondNet& net, int chi, int d, const double* A, double tol,
                 double* Pc, double* Qc, double* lam_out, double* Aout) {
  const size_t cc = (size_t)chi * chi, cdc = (size_t)chi * d * chi;
  const size_t mark = ctx->arena_off;  // consumed in stream order
  double* P = ws_alloc<double>(ctx, 2 * cc);
  double* Q = ws_alloc<double>(ctx, 2 * cc);
  double* lam = ws_alloc<double>(ctx, 2 * (size_t)chi);
  double* vw = ws_alloc<double>(ctx, 4 * cc);
  double* err = ws_alloc<double>(ctx, 1);
  double* sc = ws_alloc<double>(ctx, 2 * cdc);
  if (!sc) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted (canonical form)");
  TN_HIP(ctx, hipMemsetAsync(err, 0, sizeof(double), ctx->stream));
  {
    const size_t m2 = ctx->arena_off;
    int it = 0;
    TN_TRY(bond_truncations(ctx, chi, chi, d, A, vw, 0, tol, P, Q, lam, err, &it));
    ctx->arena_off = m2;
  }
  TN_TRY(canonical_pq(ctx, 2, chi, P, Q, Pc, Qc));
  if (lam_out)
    TN_HIP(ctx, hipMemcpyAsync(lam_out, lam, 2 * (size_t)chi * sizeof(double),
                               hipMemcpyDeviceToDevice, ctx->stream));
  TN_TRY(bondnet_truncate(ctx, net, chi, chi, A, Pc, Qc, Aout, sc));
  ctx->arena_off = mark;
  return TN_OK;
}

// out[i][s][j] = sum Q[i][a] th[a][s][b] P[b][j]   (chi x d x chi)
int sandwich(tn_ctx* ctx, int n, int chi, int d, const double* Q, const double* th, const double* P,
             double* tmp, double* out) {
  TN_TRY(gemm(ctx, chi, d * n, n, Q, n, false, th, d * n, false, tmp, d * n, 1.0, 0.0));
  TN_TRY(gemm(ctx, chi * d, chi, n, tmp, n, false, P, chi, false, out, chi, 1.0, 0.0));
  return TN_OK;
}

// two-site RDMs of the A-form chain and the TFIM energy per site
int energy_1d(tn_ctx* ctx, int chi, int d, const double* A /*[2][chi][d][chi]*/, double J,
              double h, double* e_dev) {
  const size_t cdc = (size_t)chi * d * chi, cc = (size_t)chi * chi;
  double* cell = ws_alloc<double>(ctx, 2 * cdc);
  double* v2 = ws_alloc<double>(ctx, 2 * cc);
  double* ed = ws_alloc<double>(ctx, 2);
  int* itd = ws_alloc<int>(ctx, 2);
  double* Mt = ws_alloc<double>(ctx, (size_t)chi * d * d * chi);
  double* W1 = ws_alloc<double>(ctx, (size_t)chi * d * d * chi);
  double* W2 = ws_alloc<double>(ctx, (size_t)chi * d * d * chi);
  double* rho = ws_alloc<double>(ctx, 2 * 16);
  if (!rho) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted (energy)");
  if (d != 2) TN_FAIL(ctx, TN_EINVAL, "the TFIM energy needs d = 2");
  for (int b = 0; b < 2; ++b) {
    const double* a = A + b * cdc;
    const double* c = A + (1 - b) * cdc;
    // cell [a, c]: left environment just before a, right one just after c
    TN_HIP(ctx, hipMemcpyAsync(cell, a, cdc * 8, hipMemcpyDeviceToDevice, ctx->stream));
    TN_HIP(ctx, hipMemcpyAsync(cell + cdc, c, cdc * 8, hipMemcpyDeviceToDevice, ctx->stream));
    TN_TRY(tm_pair(ctx, 2, chi, d, cell, cell, v2, ed, itd, 1e-14, 200000, 0));
    // M[x][s][t][c] = sum_b a[x][s][b] c[b][t][c]
    TN_TRY(gemm(ctx, chi * d, d * chi, chi, a, chi, false, c, d * chi, false, Mt, d * chi, 1.0,
                0.0));
    // W1[y][(s t c)] = sum_x vl[x][y] M[x][(s t c)]
    TN_TRY(gemm(ctx, chi, d * d * chi, chi, v2, chi, true, Mt, d * d * chi, false, W1,
                d * d * chi, 1.0, 0.0));
    // W2[(y s t)][e] = sum_c W1[(y s t)][c] vr[c][e]
    TN_TRY(gemm(ctx, chi * d * d, chi, chi, W1, chi, false, v2 + cc, chi, false, W2, chi, 1.0, 0.0));
    // rho[(s t)][(u v)] = sum_{y,e} W2[y][(s t)][e] M[y][(u v)][e]
    Contraction k;
    k.am = grp({{d * d, chi}});
    k.ak = grp({{chi, (long long)d * d * chi}, {chi, 1}});
    k.bk = grp({{chi, (long long)d * d * chi}, {chi, 1}});
    k.bn = grp({{d * d, chi}});
    k.cm = grp({{d * d, d * d}});
    k.cn = grp({{d * d, 1}});
    TN_TRY(tc_run(ctx, k, W2, Mt, rho + 16 * b, 1.0, 0.0));
  }
  hipLaunchKernelGGL(tfim1d_energy_kernel, dim3(1), dim3(1), 0, ctx->stream, rho, rho + 16, J, h,
                     e_dev);
  TN_HIP(ctx, hipGetLastError());
  return TN_OK;
}

}  // namespace

namespace {

// The map A_X -> G A_X of both sites as dense matrices (Sec. V B (iii)):
// G_X[(i s j)][(a t b)] = sum_{k k'} Lf_X[i][(a k)] g[k][k'][s][t] Rf_X[(b k')][j],
// site 0 with Lf[1], Rf[0], site 1 with Lf[0], Rf[1]; Gm [2][N][N], N = chi d chi.
__global__ void gate_matrix_kernel(int chi, int d, int kap, const double* __restrict__ Lf,
                                   const double* __restrict__ Rf, const double* __restrict__ g,
                                   double* __restrict__ Gm) {
  const long long N = (long long)chi * d * chi, n = (long long)kap * chi;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * N * N) return;
  const int X = (int)(t / (N * N));
  const long long e = t % (N * N), row = e / N, col = e % N;
  const int i = (int)(row / (d * chi)), s = (int)((row / chi) % d), j = (int)(row % chi);
  const int a = (int)(col / (d * chi)), tt = (int)((col / chi) % d), b = (int)(col % chi);
  const double* lf = Lf + (X == 0 ? 1 : 0) * chi * n;
  const double* rf = Rf + (X == 0 ? 0 : 1) * n * chi;
  double acc = 0.0;
  for (int k = 0; k < kap; ++k)
    for (int k2 = 0; k2 < kap; ++k2)
      acc += lf[(long long)i * n + a * kap + k] * g[((k * kap + k2) * d + s) * d + tt] *
             rf[(long long)(b * kap + k2) * chi + j];
  Gm[t] = acc;
}

// Per site: rho = v.Gv, r = |Gv - rho v| / |Gv| (v of unit norm), and the
// sign that gives v a positive overlap with the current site a; one block
// per site.
__global__ __launch_bounds__(256) void eig_residual_kernel(int N, const double* __restrict__ v,
                                                           const double* __restrict__ Gv,
                                                           const double* __restrict__ a,
                                                           double* __restrict__ out) {
  __shared__ double red[4][3];
  const int X = blockIdx.x;
  const double* vx = v + (long long)X * N;
  const double* gx = Gv + (long long)X * N;
  const double* ax = a + (long long)X * N;
  double p = 0.0, q = 0.0, o = 0.0;
  for (int e = threadIdx.x; e < N; e += 256) {
    p += vx[e] * gx[e];
    q += gx[e] * gx[e];
    o += vx[e] * ax[e];
  }
  for (int k = 32; k > 0; k >>= 1) {
    p += __shfl_xor(p, k, 64);
    q += __shfl_xor(q, k, 64);
    o += __shfl_xor(o, k, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6][0] = p;
    red[threadIdx.x >> 6][1] = q;
    red[threadIdx.x >> 6][2] = o;
  }
  __syncthreads();
  const double rho = red[0][0] + red[1][0] + red[2][0] + red[3][0];
  const double gg = red[0][1] + red[1][1] + red[2][1] + red[3][1];
  const double ov = red[0][2] + red[1][2] + red[2][2] + red[3][2];
  double r = 0.0;
  for (int e = threadIdx.x; e < N; e += 256) {
    const double z = gx[e] - rho * vx[e];
    r += z * z;
  }
  for (int k = 32; k > 0; k >>= 1) r += __shfl_xor(r, k, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][0] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double rr = red[0][0] + red[1][0] + red[2][0] + red[3][0];
    out[3 * X] = rho;
    out[3 * X + 1] = gg > 0.0 ? sqrt(rr / gg) : INFINITY;
    out[3 * X + 2] = ov < 0.0 ? -1.0 : 1.0;
  }
}

// x[X] *= sgn[3 X + 2]
__global__ void apply_sign_kernel(int N, double* __restrict__ x, const double* __restrict__ info) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2LL * N) return;
  x[t] *= info[3 * (t / N) + 2];
}

}  // namespace

namespace {

// Normalised fidelity of a two-site cell with one orthogonal U per bond,
// a_new_X ~ U[left] a_ref_X U[right]^T (site 0 has bond 1 on its left and
// bond 0 on its right): out = sum_X <a_new_X, U a_ref_X U^T> /
// sum_X |a_ref_X| |a_new_X| (one workgroup).
__global__ __launch_bounds__(256) void fidelity_1d_kernel(int chi, int d,
                                                          const double* __restrict__ a_ref,
                                                          const double* __restrict__ a_new,
                                                          const double* __restrict__ U,
                                                          double* __restrict__ out) {
  __shared__ double red[4][5];
  const long long cdc = (long long)chi * d * chi, cc = (long long)chi * chi;
  double f = 0.0, r0 = 0.0, r1 = 0.0, n0 = 0.0, n1 = 0.0;
  for (long long t = threadIdx.x; t < 2 * cdc; t += 256) {
    const int X = (int)(t / cdc);
    const long long e = t % cdc;
    const int i = (int)(e / (d * chi)), sph = (int)((e / chi) % d), j = (int)(e % chi);
    const double* Ul = U + (X == 0 ? 1 : 0) * cc;
    const double* Ur = U + (X == 0 ? 0 : 1) * cc;
    const double* ar = a_ref + X * cdc;
    double v = 0.0;
    for (int a = 0; a < chi; ++a) {
      double w = 0.0;
      for (int b = 0; b < chi; ++b) w += ar[((long long)a * d + sph) * chi + b] * Ur[j * chi + b];
      v += Ul[i * chi + a] * w;
    }
    const double an = a_new[X * cdc + e], rr = ar[e];
    f += an * v;
    if (X == 0) {
      r0 += rr * rr;
      n0 += an * an;
    } else {
      r1 += rr * rr;
      n1 += an * an;
    }
  }
  double vals[5] = {f, r0, r1, n0, n1};
  for (int q = 0; q < 5; ++q) {
    for (int o = 32; o > 0; o >>= 1) vals[q] += __shfl_xor(vals[q], o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = vals[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[5];
    for (int q = 0; q < 5; ++q) t[q] = red[0][q] + red[1][q] + red[2][q] + red[3][q];
    out[0] = t[0] / (sqrt(t[1]) * sqrt(t[3]) + sqrt(t[2]) * sqrt(t[4]));
  }
}

// U <- -U (the second bond's factor)
__global__ void negate_kernel(double* __restrict__ x, long long n) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) x[t] = -x[t];
}

// The direct method (Sec. III B 1, Eq. (iMPSDM1)) on arena memory: per bond
// the dominant left eigenvector X of the mixed transfer matrix of a_ref
// (ket) and a_new (bra) is w U^T for a positive w, so U is the orthogonal
// polar factor of X^T; the overall sign of the pair (U0, U1) is taken with
// F > 0.  *itmax: the larger fixed-point iteration count of the two bonds.
int gauge_direct_1d(tn_ctx* ctx, int chi, int d, const double* a_ref, const double* a_new,
                    double* U, double tol, int max_iter, double* fidelity, int* itmax_out) {
  const size_t cdc = (size_t)chi * d * chi, cc = (size_t)chi * chi;
  double* kets = ws_alloc<double>(ctx, 4 * cdc);
  double* bras = ws_alloc<double>(ctx, 4 * cdc);
  double* v4 = ws_alloc<double>(ctx, 4 * cc);
  double* W = ws_alloc<double>(ctx, 2 * cc);
  double* V = ws_alloc<double>(ctx, 2 * cc);
  double* S = ws_alloc<double>(ctx, 2 * (size_t)chi);
  double* ed = ws_alloc<double>(ctx, 4);
  int* itd = ws_alloc<int>(ctx, 4);
  double* fd = ws_alloc<double>(ctx, 2);
  if (!fd) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted (1D gauge fix)");
  // the cell of bond b ends with the site left of it: [ref 1, ref 0] for
  // bond 0, [ref 0, ref 1] for bond 1 (bras likewise); both bonds in one
  // launch, their left fixed points at v4[0] and v4[2]
  for (int b = 0; b < 2; ++b) {
    const int a = b == 0 ? 0 : 1, c = 1 - a;
    TN_HIP(ctx, hipMemcpyAsync(kets + 2 * b * cdc, a_ref + c * cdc, cdc * 8,
                               hipMemcpyDeviceToDevice, ctx->stream));
    TN_HIP(ctx, hipMemcpyAsync(kets + (2 * b + 1) * cdc, a_ref + a * cdc, cdc * 8,
                               hipMemcpyDeviceToDevice, ctx->stream));
    TN_HIP(ctx, hipMemcpyAsync(bras + 2 * b * cdc, a_new + c * cdc, cdc * 8,
                               hipMemcpyDeviceToDevice, ctx->stream));
    TN_HIP(ctx, hipMemcpyAsync(bras + (2 * b + 1) * cdc, a_new + a * cdc, cdc * 8,
                               hipMemcpyDeviceToDevice, ctx->stream));
  }
  {
    const size_t mark = ctx->arena_off;
    TN_TRY(tm_pair(ctx, 2, chi, d, kets, bras, v4, ed, itd, tol > 0 ? tol : 1e-14, max_iter, 0,
                   nullptr, true, 2));
    ctx->arena_off = mark;
  }
  // the polar factor of X^T: with X = W S V^T (X^T = V S W^T), U = V W^T
  TN_TRY(jacobi_svd(ctx, 2, chi, chi, v4, chi, 2 * (long long)cc, W, chi, (long long)cc, S, chi,
                    V, chi, (long long)cc));
  TN_TRY(gemm(ctx, chi, chi, chi, V, chi, false, W, chi, true, U, chi, 1.0, 0.0, 2, (long long)cc,
              (long long)cc, (long long)cc));
  int hi[4];
  TN_HIP(ctx, hipMemcpyAsync(hi, itd, 4 * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  const int itmax = std::max(std::max(hi[0], hi[1]), std::max(hi[2], hi[3]));
  hipLaunchKernelGGL(fidelity_1d_kernel, dim3(1), dim3(256), 0, ctx->stream, chi, d, a_ref, a_new,
                     U, fd);
  TN_HIP(ctx, hipGetLastError());
  TN_HIP(ctx, hipMemcpyAsync(ctx->host_scratch, fd, sizeof(double), hipMemcpyDeviceToHost,
                             ctx->stream));
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  double F = ctx->host_scratch[0];
  if (F < 0) {
    hipLaunchKernelGGL(negate_kernel, dim3((unsigned)((cc + 255) / 256)), dim3(256), 0,
                       ctx->stream, U + cc, (long long)cc);
    TN_HIP(ctx, hipGetLastError());
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
    F = -F;
  }
  if (!std::isfinite(F)) TN_FAIL(ctx, TN_ENUMERIC, "non-finite fidelity");
  if (fidelity) *fidelity = F;
  if (itmax_out) *itmax_out = itmax;
  return TN_OK;
}

// Arena bytes gauge_direct_1d needs beyond the caller's.
size_t gauge_direct_bytes(int chi, int d) {
  const size_t cdc = (size_t)chi * d * chi, cc = (size_t)chi * chi;
  const size_t tmw = tm_work_in_global(2, chi, d) ? 4 * tm_work_per_side(2, chi, d) : 0;
  // cells, fixed points, SVD factors, the four sides' Krylov bases
  return (8 * cdc + 10 * cc + 4 * (TM_KRYLOV + 1) * cc + tmw + 64) * 8 + (1 << 20);
}

}  // namespace

// Gauge fixing of a two-site iMPS (Sec. III B): a_new ~ U a_ref U^T per
// site with one orthogonal U per bond (U [2][chi][chi], bond 0 after site
// 0).  method 0: the iterative method (Sec. III B 2, Eq. (15)), alternating
// Procrustes steps from the U passed in until F changes by less than tol;
// method 1: the direct method (gauge_direct_1d).
int gauge_fix_1d(tn_ctx* ctx, int method, int chi, int d, const double* a_ref,
                 const double* a_new, double* U, double tol, int max_iter, double* fidelity,
                 int* iters) {
  if (chi < 1 || d < 1 || !a_ref || !a_new || !U || max_iter < 1)
    TN_FAIL(ctx, TN_EINVAL, "bad 1D gauge_fix arguments");
  if (chi > TN_SMALL_BOND)
    TN_FAIL(ctx, TN_EINVAL, "1D gauge fixing supports chi <= %d (chi=%d)", TN_SMALL_BOND, chi);
  const BondNet net = bondnet_chain2(d);
  TN_TRY(ws_reserve(ctx, bondnet_gauge_bytes(net, chi) + gauge_direct_bytes(chi, d)));
  ws_reset(ctx);
  if (method == 0)
    return bondnet_gauge_fix(ctx, net, chi, a_ref, a_new, U, tol, max_iter, fidelity, iters);
  if (method != 1) TN_FAIL(ctx, TN_EINVAL, "unknown 1D gauge-fix method %d", method);
  int itmax = 0;
  TN_TRY(gauge_direct_1d(ctx, chi, d, a_ref, a_new, U, tol, max_iter, fidelity, &itmax));
  if (iters) *iters = itmax;
  return itmax >= max_iter ? TN_NOT_CONVERGED : TN_OK;
}

// N_Re -> infinity (Sec. V C): each site becomes the dominant eigenvector of
// its renormalized gate.  The dense map G_X is squared with normalisation,
// M <- M M / |M M|_F, which converges to the projector on the dominant
// eigenvector (a power method that doubles the power per step); after each
// squaring v = M a / |M a| is tested for G v = rho v.  Returns TN_OK,
// TN_NOT_CONVERGED (no simple real dominant eigenvalue within 2^60 powers).
int recycle_limit(tn_ctx* ctx, int chi, int d, int kap, const double* Lf, const double* Rf,
                  const double* g, double* A, double* rho_out) {
  const int N = chi * d * chi;
  const size_t NN = (size_t)N * N;
  double* Gm = ws_alloc<double>(ctx, 2 * NN);
  double* M = ws_alloc<double>(ctx, 2 * NN);
  double* M2 = ws_alloc<double>(ctx, 2 * NN);
  double* v = ws_alloc<double>(ctx, 2 * (size_t)N);
  double* Gv = ws_alloc<double>(ctx, 2 * (size_t)N);
  double* info = ws_alloc<double>(ctx, 8);
  if (!info) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted (recycling limit)");
  hipLaunchKernelGGL(gate_matrix_kernel, dim3((unsigned)((2 * NN + 255) / 256)), dim3(256), 0,
                     ctx->stream, chi, d, kap, Lf, Rf, g, Gm);
  TN_HIP(ctx, hipGetLastError());
  for (int X = 0; X < 2; ++X) TN_TRY(frob_normalize_to(ctx, Gm + X * NN, M + X * NN, NN, nullptr));
  double res = INFINITY, prev = INFINITY;
  int sq = 0;
  for (sq = 1; sq <= 60; ++sq) {
    TN_TRY(gemm(ctx, N, N, N, M, N, false, M, N, false, M2, N, 1.0, 0.0, 2, (long long)NN,
                (long long)NN, (long long)NN));
    for (int X = 0; X < 2; ++X) TN_TRY(frob_normalize_to(ctx, M2 + X * NN, M + X * NN, NN, nullptr));
    // v = M a / |M a|, then G v and the residual
    TN_TRY(gemm(ctx, N, 1, N, M, N, false, A, 1, false, v, 1, 1.0, 0.0, 2, (long long)NN,
                (long long)N, (long long)N));
    for (int X = 0; X < 2; ++X) TN_TRY(frob_normalize(ctx, v + X * N, N, nullptr));
    TN_TRY(gemm(ctx, N, 1, N, Gm, N, false, v, 1, false, Gv, 1, 1.0, 0.0, 2, (long long)NN,
                (long long)N, (long long)N));
    hipLaunchKernelGGL(eig_residual_kernel, dim3(2), dim3(256), 0, ctx->stream, N, v, Gv, A,
                       info);
    TN_HIP(ctx, hipGetLastError());
    TN_HIP(ctx, hipMemcpyAsync(ctx->host_scratch, info, 6 * sizeof(double),
                               hipMemcpyDeviceToHost, ctx->stream));
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
    prev = res;
    res = std::max(ctx->host_scratch[1], ctx->host_scratch[4]);
    if (!std::isfinite(res)) TN_FAIL(ctx, TN_ENUMERIC, "non-finite renormalized-gate eigenvector");
    // converged, or at the rounding floor
    if (res < 1e-13 || (res < 1e-10 && res > 0.5 * prev)) break;
  }
  if (rho_out) {
    rho_out[0] = ctx->host_scratch[0];
    rho_out[1] = ctx->host_scratch[3];
  }
  hipLaunchKernelGGL(apply_sign_kernel, dim3((unsigned)((2LL * N + 255) / 256)), dim3(256), 0,
                     ctx->stream, N, v, info);
  TN_HIP(ctx, hipGetLastError());
  TN_HIP(ctx, hipMemcpyAsync(A, v, 2 * (size_t)N * sizeof(double), hipMemcpyDeviceToDevice,
                             ctx->stream));
  return res < 1e-10 ? TN_OK : TN_NOT_CONVERGED;
}

namespace {

// The scalar a step reports for its new state: the TFIM energy per site, or
// ln Z per site of the classical model whose row transfer matrix the gate is.
struct StepMeasure {
  int kind;  // 0: TFIM energy (J, h), 1: classical ln Z (beta)
  double J, h, beta;
};

__global__ void pad_bra_kernel(const double* __restrict__ A, double* __restrict__ B, int chi,
                               int d, int kap) {
  // B[(i, a)][s][(j, b)] = A[i][s][j] for a = b = 0, else 0 (two sites)
  const int n = chi * kap;
  const long long tot = 2LL * n * d * n;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= tot) return;
  long long r = t;
  const int jb = r % n; r /= n;
  const int s = r % d; r /= d;
  const int ia = r % n; r /= n;
  const int site = (int)r;
  B[t] = (ia % kap == 0 && jb % kap == 0)
             ? A[(((long long)site * chi + ia / kap) * d + s) * chi + jb / kap]
             : 0.0;
}

__global__ void log_z_kernel(const double* __restrict__ eta1, const double* __restrict__ eta0,
                             double log_scale, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0)
    out[0] = log_scale + 0.5 * (log(eta1[0]) - log(eta0[0]));
}

// ln Z per site of the classical Ising model from the two-site iMPS A:
// ln c + ln mu, mu the per-site Rayleigh quotient of the gate g, i.e. the
// square root of the ratio of the dominant eigenvalues of the mixed
// transfer matrix of (g A, A) (A zero-padded to the bond kappa chi) and of
// (A, A) over the cell.
int log_z_1d(tn_ctx* ctx, int chi, int d, int kap, const double* A, const double* g,
             double log_scale, double* out_dev) {
  const int n = kap * chi;
  const size_t ndn = (size_t)n * d * n, cdc = (size_t)chi * d * chi;
  double* th = ws_alloc<double>(ctx, 2 * ndn);
  double* bp = ws_alloc<double>(ctx, 2 * ndn);
  double* v2 = ws_alloc<double>(ctx, 2 * (size_t)n * n);
  double* ed = ws_alloc<double>(ctx, 4);
  int* itd = ws_alloc<int>(ctx, 4);
  if (!itd) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted (ln Z)");
  for (int s = 0; s < 2; ++s)
    hipLaunchKernelGGL(impo_apply_kernel, dim3((unsigned)((ndn + 255) / 256)), dim3(256), 0,
                       ctx->stream, g, A + s * cdc, th + s * ndn, chi, d, kap);
  hipLaunchKernelGGL(pad_bra_kernel, dim3((unsigned)((2 * ndn + 255) / 256)), dim3(256), 0,
                     ctx->stream, A, bp, chi, d, kap);
  TN_HIP(ctx, hipGetLastError());
  TN_TRY(tm_pair(ctx, 2, n, d, th, bp, v2, ed, itd, 1e-14, 200000, 0));
  TN_TRY(tm_pair(ctx, 2, chi, d, A, A, v2, ed + 2, itd + 2, 1e-14, 200000, 0));
  hipLaunchKernelGGL(log_z_kernel, dim3(1), dim3(64), 0, ctx->stream, ed, ed + 2, log_scale,
                     out_dev);
  TN_HIP(ctx, hipGetLastError());
  return TN_OK;
}

int step_measure(tn_ctx* ctx, int chi, int d, const double* A, const double* g,
                 const StepMeasure& m, double* out_dev) {
  if (m.kind == 0) return energy_1d(ctx, chi, d, A, m.J, m.h, out_dev);
  return log_z_1d(ctx, chi, d, 2, A, g, 0.5 * log(2.0 * sinh(2.0 * m.beta)), out_dev);
}

// One step of the power method with the two-site iMPO hg (iTEBD, Sec. V):
// the modes of itebd_step, and the measurement m of the new state into
// *meas_or_null.
int itebd_core(tn_ctx* ctx, int chi, int d, double* A /*[2][chi][d][chi] in/out*/,
               const double hg[2][2][2][2], const StepMeasure& meas, int mode, double* env1d,
               double* lambda_out, double tol, double* trunc_err, double* energy_or_null) {
  if (chi < 1 || d != 2 || !A || !env1d) TN_FAIL(ctx, TN_EINVAL, "bad itebd_step arguments");
  if (mode < 0 || mode > 4) TN_FAIL(ctx, TN_EINVAL, "itebd_step mode %d not available", mode);
  // mode 4 is the environment step of mode 1 with the direct gauge fix
  const bool direct = mode == 4;
  if (direct) mode = 1;
  const int kap = 2, n = kap * chi;
  if (mode != 0 && chi > TN_SMALL_BOND)
    TN_FAIL(ctx, TN_EINVAL, "recycling supports chi <= %d (chi=%d)", TN_SMALL_BOND, chi);
  const size_t nn = (size_t)n * n, ndn = (size_t)n * d * n, cdc = (size_t)chi * d * chi;
  const size_t cc = (size_t)chi * chi;
  const BondNet net = bondnet_chain2(d);
  size_t extra = 0;
  if (mode == 1)
    extra = bondnet_canon_bytes(net, chi) + bondnet_gauge_bytes(net, chi) +
            (direct ? gauge_direct_bytes(chi, d) : 0) + (12 * cc + 4 * cdc) * 8;
  if (mode == 3) extra = (6 * cdc * cdc + 4 * cdc + 64) * 8;
  if (energy_or_null && meas.kind == 1)
    extra += (4 * ndn + 2 * nn + 8) * 8 + 2 * tm_work_per_side(2, n, d) * 8;
  // the batched truncation: Krylov bases and fixed-point workspaces of four
  // sides, four factor SVDs and two bond SVDs
  const size_t tmw = tm_work_in_global(2, n, d) ? 4 * tm_work_per_side(2, n, d) : 0;
  TN_TRY(ws_reserve(ctx, (96 * nn + 12 * ndn + 16 * cdc + tmw) * 8 + extra + (8 << 20)));
  ws_reset(ctx);
  double* g = ws_alloc<double>(ctx, 16);
  double* th = ws_alloc<double>(ctx, 2 * ndn);
  double* P = ws_alloc<double>(ctx, 2 * (size_t)n * chi);
  double* Q = ws_alloc<double>(ctx, 2 * (size_t)n * chi);
  double* lam = ws_alloc<double>(ctx, 2 * (size_t)chi);
  double* errd = ws_alloc<double>(ctx, 1);
  double* edev = ws_alloc<double>(ctx, 1);
  double* tmp = ws_alloc<double>(ctx, (size_t)chi * d * n);
  if (!tmp) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted (itebd)");
  TN_HIP(ctx, hipMemcpyAsync(g, hg, 16 * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  TN_HIP(ctx, hipMemsetAsync(errd, 0, sizeof(double), ctx->stream));
  // env1d: warm fixed points [4 n^2], the renormalized gate's factors
  // Lf [2][chi][n] and Rf [2][n][chi], then flags: slot 0 marks the fixed
  // points valid, slot 1 the factors
  double* Lf = env1d + 4 * nn;
  double* Rf = Lf + 2 * (size_t)chi * n;
  double* flagp = env1d + env1d_doubles(chi, d) - 16;
  double hflag[2] = {0.0, 0.0};
  TN_HIP(ctx, hipMemcpyAsync(hflag, flagp, 2 * sizeof(double), hipMemcpyDeviceToHost,
                             ctx->stream));
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  auto gate = [&](const double* src) -> int {
    for (int s = 0; s < 2; ++s)
      hipLaunchKernelGGL(impo_apply_kernel, dim3((unsigned)((ndn + 255) / 256)), dim3(256), 0,
                         ctx->stream, g, src + s * cdc, th + s * ndn, chi, d, kap);
    TN_HIP(ctx, hipGetLastError());
    return TN_OK;
  };
  // site 0 sits between bond 1 (left) and bond 0 (right), site 1 the reverse:
  // dst_0 = L[1] th_0 R[0], dst_1 = L[0] th_1 R[1], each of unit norm
  auto truncate2 = [&](const double* Lm, const double* Rm, double* dst) -> int {
    TN_TRY(sandwich(ctx, n, chi, d, Lm + 1 * n * chi, th, Rm, tmp, dst));
    TN_TRY(sandwich(ctx, n, chi, d, Lm, th + ndn, Rm + 1 * n * chi, tmp, dst + cdc));
    TN_TRY(frob_normalize(ctx, dst, cdc, nullptr));
    TN_TRY(frob_normalize(ctx, dst + cdc, cdc, nullptr));
    return TN_OK;
  };
  if (mode == 2 || mode == 3) {
    // recycled step: A <- G A with the stored factors (Sec. V B), or its
    // limit N_Re -> infinity, the dominant eigenvector of G (Sec. V C)
    if (hflag[1] != 1.0)
      TN_FAIL(ctx, TN_EINVAL, "no renormalized gate in env1d: run a TN_RECYCLE_BUILD step first");
    int rc = TN_OK;
    if (mode == 2) {
      TN_TRY(gate(A));
      TN_TRY(truncate2(Lf, Rf, A));
    } else {
      rc = recycle_limit(ctx, chi, d, kap, Lf, Rf, g, A, nullptr);
      if (rc < 0) return rc;
    }
    if (energy_or_null) {
      TN_TRY(step_measure(ctx, chi, d, A, g, meas, edev));
      double he = 0.0;
      TN_HIP(ctx, hipMemcpyAsync(&he, edev, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
      TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
      *energy_or_null = he;
    } else {
      TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    if (trunc_err) *trunc_err = 0.0;
    return rc;
  }
  double* a0 = A;  // the state the environment is computed for
  double *a0c = nullptr, *tr = nullptr, *Pc = nullptr, *Qc = nullptr, *U = nullptr,
         *l1 = nullptr, *a1 = nullptr;
  if (mode == 1) {
    a0c = ws_alloc<double>(ctx, 2 * cdc);
    tr = ws_alloc<double>(ctx, 2 * cdc);
    a1 = ws_alloc<double>(ctx, 2 * cdc);
    Pc = ws_alloc<double>(ctx, 2 * cc);
    Qc = ws_alloc<double>(ctx, 2 * cc);
    U = ws_alloc<double>(ctx, 2 * cc);
    l1 = ws_alloc<double>(ctx, 2 * (size_t)chi);
    if (!l1) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted (recycling)");
    // the scheme starts from the canonical form of A_0 (Sec. V B (i))
    const size_t mark = ctx->arena_off;
    TN_TRY(canonical_1d(ctx, net, chi, d, A, tol, Pc, Qc, nullptr, a0c));
    ctx->arena_off = mark;
    a0 = a0c;
  }
  TN_TRY(gate(a0));
  const int warm = hflag[0] == 1.0 ? 1 : 0;
  int tmi = 0;
  {
    const size_t mark = ctx->arena_off;
    TN_TRY(bond_truncations(ctx, n, chi, d, th, env1d, warm, tol, P, Q, lam, errd, &tmi));
    ctx->arena_off = mark;
  }
  const double one = 1.0;
  TN_HIP(ctx, hipMemcpyAsync(flagp, &one, sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  if (mode == 0) {
    TN_TRY(truncate2(Q, P, A));
    if (lambda_out)
      TN_HIP(ctx, hipMemcpyAsync(lambda_out, lam, 2 * chi * sizeof(double),
                                 hipMemcpyDeviceToDevice, ctx->stream));
  } else {
    // truncated state, its canonical form, gauge fix against A_0 and the
    // renormalized gate G = U^T (Qc Q) g (P Pc) U (Sec. V B (i)-(iii))
    TN_TRY(truncate2(Q, P, tr));
    size_t mark = ctx->arena_off;
    TN_TRY(canonical_1d(ctx, net, chi, d, tr, tol, Pc, Qc, l1, a1));
    ctx->arena_off = mark;
    double F = 0.0;
    if (direct) {
      int it = 0;
      TN_TRY(gauge_direct_1d(ctx, chi, d, a0c, a1, U, tol, 100000, &F, &it));
      tmi = it > tmi ? it : tmi;
    } else {
      TN_TRY(recycle_gauge_start(ctx, 2, n, chi, kap, P, Q, Pc, Qc, U));
      const int rc = bondnet_gauge_fix(ctx, net, chi, a0c, a1, U, 1e-12, 1000, &F, nullptr);
      if (rc < 0) return rc;
    }
    ctx->arena_off = mark;
    TN_TRY(recycle_factors(ctx, 2, n, chi, P, Q, Pc, Qc, U, Rf, Lf));
    TN_HIP(ctx, hipMemcpyAsync(flagp + 1, &one, sizeof(double), hipMemcpyHostToDevice,
                               ctx->stream));
    // the new state is G A_0
    TN_TRY(truncate2(Lf, Rf, A));
    if (lambda_out)
      TN_HIP(ctx, hipMemcpyAsync(lambda_out, l1, 2 * chi * sizeof(double),
                                 hipMemcpyDeviceToDevice, ctx->stream));
  }
  if (energy_or_null) TN_TRY(step_measure(ctx, chi, d, A, g, meas, edev));
  double he = 0.0, herr = 0.0;
  TN_HIP(ctx, hipMemcpyAsync(&herr, errd, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  if (energy_or_null)
    TN_HIP(ctx, hipMemcpyAsync(&he, edev, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (trunc_err) *trunc_err = herr;
  if (energy_or_null) *energy_or_null = he;
  if (!std::isfinite(herr)) TN_FAIL(ctx, TN_ENUMERIC, "non-finite truncation");
  return tmi >= 100000 ? TN_NOT_CONVERGED : TN_OK;
}

}  // namespace

int itebd_step_impl(tn_ctx* ctx, int chi, int d, double* A, double J, double h, double dt,
                    int mode, double* env1d, double* lambda_out, double tol, double* trunc_err,
                    double* energy_or_null) {
  double hg[2][2][2][2];
  tfim_impo(J, h, dt, hg);
  return itebd_core(ctx, chi, d, A, hg, StepMeasure{0, J, h, 0.0}, mode, env1d, lambda_out, tol,
                    trunc_err, energy_or_null);
}

// The row transfer matrix of the square-lattice Ising model (J = 1, inverse
// temperature beta) is c^L times the second-order TFIM gate at dt J = beta,
// dt h = K* (tanh K* = exp(-2 beta)), c = sqrt(2 sinh 2 beta): one power-
// method step on it is an iTEBD step with that gate (Sec. I).
int ising2d_tm_step_impl(tn_ctx* ctx, int chi, double* A, double beta, int mode, double* env1d,
                         double* lambda_out, double tol, double* trunc_err, double* lnz_or_null) {
  if (!(beta > 0.0) || !std::isfinite(beta))
    TN_FAIL(ctx, TN_EINVAL, "inverse temperature %g must be positive", beta);
  const double kstar = atanh(exp(-2.0 * beta));
  double hg[2][2][2][2];
  tfim_impo(beta, kstar, 1.0, hg);
  return itebd_core(ctx, chi, 2, A, hg, StepMeasure{1, 0.0, 0.0, beta}, mode, env1d,
                    lambda_out, tol, trunc_err, lnz_or_null);
}
