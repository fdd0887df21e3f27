// Full update of an iPEPS with environment recycling (Sec. VI B, VI C of the
// paper), the canonical form of an iPEPS (Sec. IV A) and gauge fixing
// (Sec. IV B, Eq. (25)) on the GPU.
//
// Site tensors here are small (d (kappa D)^4 entries), so the elementwise and
// per-leg kernels are plain one-pass kernels over L2-resident data and the
// small factorisations run one workgroup per matrix.  The bond environment N
// of a link -- the CTM network around the link's two sites with the link's
// ket and bra legs open -- is the one sizeable contraction and runs on the
// table-driven MFMA contraction engine, as two half networks joined over
// their boundary legs.
//
// Links of a unit cell are enumerated in first-seen order over the positions
// (p = y Lx + x), the right link of a position before its down link; link b
// joins leg l1 (r or d) of site s1 to leg l2 (l or u) of site s2.  On a link
// the first site carries P (new = P^T old on that leg) and the second Q
// (new = Q old), as in A~ = Q Theta P.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <vector>

#include "bondnet.h"
#include "common.h"

int ipeps_rdms_impl(tn_ctx* ctx, int Lx, int Ly, int D, int d, int nsite, const double* sites,
                    const int* cell, int chi, const double* C, const double* T, double* rho1,
                    double* rhoh, double* rhov);

namespace {

constexpr int MAXL = 64;        // links of a cell
constexpr int MAXN = TN_SMALL_BOND;  // largest bond handled by the small per-leg kernels
// entries of an n x n result per thread of a 256-thread workgroup (n <= MAXN)
constexpr int EPT = (MAXN * MAXN + 255) / 256;
constexpr double CUT = 1e-14;   // relative cutoff of pseudo-inverse square roots
enum { AX_S = 0, AX_L = 1, AX_R = 2, AX_D = 3, AX_U = 4 };

// ---------------------------------------------------------------------------
// cell links
// ---------------------------------------------------------------------------

struct CellLinks {
  int nl = 0;
  int s1[MAXL], l1[MAXL], s2[MAXL], l2[MAXL];
  int x[MAXL], y[MAXL];  // position of the first site where the link is first met
  std::vector<std::array<int, 5>> leg_link;  // [site][axis] -> link
};

int build_links(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, CellLinks& L) {
  if (Lx < 1 || Ly < 1 || nsite < 1 || !cell) TN_FAIL(ctx, TN_EINVAL, "bad unit cell");
  if (Lx * Ly > 64) TN_FAIL(ctx, TN_EINVAL, "cell larger than 64 positions");
  for (int p = 0; p < Lx * Ly; ++p)
    if (cell[p] < 0 || cell[p] >= nsite)
      TN_FAIL(ctx, TN_EINVAL, "cell[%d] = %d out of range [0, %d)", p, cell[p], nsite);
  L.nl = 0;
  L.leg_link.assign(nsite, {-1, -1, -1, -1, -1});
  auto pos = [&](int x, int y) { return (((y % Ly) + Ly) % Ly) * Lx + (((x % Lx) + Lx) % Lx); };
  for (int y = 0; y < Ly; ++y)
    for (int x = 0; x < Lx; ++x) {
      const int s = cell[pos(x, y)];
      const int legs[2][4] = {{AX_R, AX_L, 1, 0}, {AX_D, AX_U, 0, 1}};
      for (auto& lg : legs) {
        const int t = cell[pos(x + lg[2], y + lg[3])];
        int b = -1;
        for (int k = 0; k < L.nl; ++k)
          if (L.s1[k] == s && L.l1[k] == lg[0] && L.s2[k] == t) b = k;
        if (b < 0) {
          if (L.nl == MAXL) TN_FAIL(ctx, TN_EINVAL, "too many links");
          b = L.nl++;
          L.s1[b] = s;
          L.l1[b] = lg[0];
          L.s2[b] = t;
          L.l2[b] = lg[1];
          L.x[b] = x;
          L.y[b] = y;
        }
        const int ends[2][2] = {{s, lg[0]}, {t, lg[1]}};
        for (auto& e : ends) {
          int& slot = L.leg_link[e[0]][e[1]];
          if (slot >= 0 && slot != b)
            TN_FAIL(ctx, TN_EINVAL, "the cell assigns two links to leg %d of site %d", e[1], e[0]);
          slot = b;
        }
      }
    }
  for (int s = 0; s < nsite; ++s)
    if (L.leg_link[s][AX_L] < 0) TN_FAIL(ctx, TN_EINVAL, "site %d does not occur in the cell", s);
  return TN_OK;
}

// ---------------------------------------------------------------------------
// tensor shapes and per-leg kernels
// ---------------------------------------------------------------------------

struct TDims {
  int n[5];
};

__host__ __device__ inline long long tsize(const TDims& t) {
  return (long long)t.n[0] * t.n[1] * t.n[2] * t.n[3] * t.n[4];
}

TDims dims5(int d, int a, int b, int c, int e) { return TDims{{d, a, b, c, e}}; }

// out = m applied on axis ax of in: out[.., i, ..] = sum_a m_eff[i][a] in[.., a, ..],
// m_eff = m (nnew x nold) or, with trans, m^T for m stored nold x nnew
__global__ void apply_leg_kernel(const double* __restrict__ in, double* __restrict__ out, TDims din,
                                 int ax, const double* __restrict__ m, int trans, int nnew) {
  TDims dout = din;
  dout.n[ax] = nnew;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= tsize(dout)) return;
  int idx[5];
  long long r = t;
  for (int k = 4; k >= 0; --k) {
    idx[k] = (int)(r % dout.n[k]);
    r /= dout.n[k];
  }
  long long st[5];
  st[4] = 1;
  for (int k = 3; k >= 0; --k) st[k] = st[k + 1] * din.n[k + 1];
  long long base = 0;
  for (int k = 0; k < 5; ++k)
    if (k != ax) base += idx[k] * st[k];
  const int i = idx[ax], nold = din.n[ax];
  double acc = 0.0;
  for (int a = 0; a < nold; ++a) {
    const double mv = trans ? m[(long long)a * nnew + i] : m[(long long)i * nold + a];
    acc += mv * in[base + a * st[ax]];
  }
  out[t] = acc;
}

int apply_leg(tn_ctx* ctx, const double* in, double* out, TDims din, int ax, const double* m,
              int trans, int nnew) {
  TDims dout = din;
  dout.n[ax] = nnew;
  const long long tot = tsize(dout);
  hipLaunchKernelGGL(apply_leg_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                     ctx->stream, in, out, din, ax, m, trans, nnew);
  TN_HIP(ctx, hipGetLastError());
  return TN_OK;
}

// One matrix per bond axis (null: leave the axis alone), applied in axis
// order; `out` receives the result, t1/t2 are scratch of the largest
// intermediate size.  Returns the output shape in *dout.
struct LegMats {
  const double* m[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int trans[5] = {0, 0, 0, 0, 0};
  int nnew[5] = {0, 0, 0, 0, 0};
};

int apply_legs(tn_ctx* ctx, const double* in, double* out, TDims din, const LegMats& lm,
               double* t1, double* t2, TDims* dout) {
  int todo[5], nt = 0;
  for (int ax = 0; ax <= 4; ++ax)
    if (lm.m[ax]) todo[nt++] = ax;
  TDims cur = din;
  const double* src = in;
  for (int k = 0; k < nt; ++k) {
    const int ax = todo[k];
    double* dst = (k == nt - 1) ? out : ((k & 1) ? t2 : t1);
    TN_TRY(apply_leg(ctx, src, dst, cur, ax, lm.m[ax], lm.trans[ax], lm.nnew[ax]));
    cur.n[ax] = lm.nnew[ax];
    src = dst;
  }
  if (nt == 0)
    TN_HIP(ctx, hipMemcpyAsync(out, in, tsize(din) * sizeof(double), hipMemcpyDeviceToDevice,
                               ctx->stream));
  if (dout) *dout = cur;
  return TN_OK;
}

// one counter-clockwise rotation: new (l, r, d, u) = old (u, d, l, r)
__global__ void rotate_kernel(const double* __restrict__ in, double* __restrict__ out, TDims din) {
  const TDims dout{{din.n[0], din.n[4], din.n[3], din.n[1], din.n[2]}};
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= tsize(dout)) return;
  long long r = t;
  const int e = (int)(r % dout.n[4]); r /= dout.n[4];
  const int c = (int)(r % dout.n[3]); r /= dout.n[3];
  const int b = (int)(r % dout.n[2]); r /= dout.n[2];
  const int a = (int)(r % dout.n[1]); r /= dout.n[1];
  const int s = (int)r;
  // new[s][a][b][c][e] = old[s][l=c][r=e][d=b][u=a]
  const long long src =
      ((((long long)s * din.n[1] + c) * din.n[2] + e) * din.n[3] + b) * din.n[4] + a;
  out[t] = in[src];
}

int rotate_times(tn_ctx* ctx, const double* in, double* out, double* tmp, TDims din, int times,
                 TDims* dout) {
  TDims cur = din;
  const double* src = in;
  if (times == 0) {
    TN_HIP(ctx, hipMemcpyAsync(out, in, tsize(din) * sizeof(double), hipMemcpyDeviceToDevice,
                               ctx->stream));
  }
  for (int k = 0; k < times; ++k) {
    // alternate so that the last rotation lands in out
    double* dst = ((times - 1 - k) & 1) ? tmp : out;
    const long long tot = tsize(cur);
    hipLaunchKernelGGL(rotate_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                       ctx->stream, src, dst, cur);
    TN_HIP(ctx, hipGetLastError());
    cur = TDims{{cur.n[0], cur.n[4], cur.n[3], cur.n[1], cur.n[2]}};
    src = dst;
  }
  if (dout) *dout = cur;
  return TN_OK;
}

// Gram-type products over every index but one bond axis:
// out[i][i'] = sum_terms sum_rest A_t[.., i, ..] w(rest) B_t[.., i', ..] w(rest)
// with the open index on axis ax[t] of term t, w(rest) = product of
// lam_k[index on axis k] over the weighted axes k (null: weight 1).
struct GramJob {
  const double* A[2];
  const double* B[2];
  int ax[2];
  int nterm;
  TDims dims;
  const double* lam[5];
  double* out;
};
constexpr int GRAM_JOBS = 16;
struct GramBatch {
  GramJob job[GRAM_JOBS];
};

constexpr int GRAM_CHUNK = 64;

__global__ __launch_bounds__(256) void leg_gram_kernel(GramBatch batch) {
  const GramJob& J = batch.job[blockIdx.x];
  const int n = J.dims.n[J.ax[0]];
  __shared__ double ta[MAXN][GRAM_CHUNK + 1], tb[MAXN][GRAM_CHUNK + 1];
  long long st[5];
  st[4] = 1;
  for (int k = 3; k >= 0; --k) st[k] = st[k + 1] * J.dims.n[k + 1];
  const long long rest = tsize(J.dims) / n;
  double acc[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) acc[q] = 0.0;
  const int tid = threadIdx.x;
  for (int term = 0; term < J.nterm; ++term) {
    const double* A = J.A[term];
    const double* B = J.B[term];
    const int ax = J.ax[term];
    int other[4], no = 0;
    for (int k = 0; k < 5; ++k)
      if (k != ax) other[no++] = k;
    for (long long c0 = 0; c0 < rest; c0 += GRAM_CHUNK) {
      for (int e = tid; e < n * GRAM_CHUNK; e += 256) {
        const int i = e / GRAM_CHUNK, c = e % GRAM_CHUNK;
        const long long col = c0 + c;
        double va = 0.0, vb = 0.0;
        if (col < rest) {
          long long r = col, off = 0;
          double w = 1.0;
          for (int q = 3; q >= 0; --q) {
            const int k = other[q];
            const int ik = (int)(r % J.dims.n[k]);
            r /= J.dims.n[k];
            off += ik * st[k];
            if (J.lam[k]) w *= J.lam[k][ik];
          }
          off += (long long)i * st[ax];
          va = A[off] * w;
          vb = B[off] * w;
        }
        ta[i][c] = va;
        tb[i][c] = vb;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const int e = tid + q * 256;
        if (e < n * n) {
          const int i = e / n, j = e % n;
          double s = 0.0;
          for (int c = 0; c < GRAM_CHUNK; ++c) s += ta[i][c] * tb[j][c];
          acc[q] += s;
        }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = tid + q * 256;
    if (e < n * n) J.out[e] = acc[q];
  }
}

int run_grams(tn_ctx* ctx, const std::vector<GramJob>& jobs) {
  for (size_t j0 = 0; j0 < jobs.size(); j0 += GRAM_JOBS) {
    GramBatch b;
    std::memset(&b, 0, sizeof(b));
    const int nj = (int)std::min<size_t>(GRAM_JOBS, jobs.size() - j0);
    for (int j = 0; j < nj; ++j) b.job[j] = jobs[j0 + j];
    hipLaunchKernelGGL(leg_gram_kernel, dim3(nj), dim3(256), 0, ctx->stream, b);
    TN_HIP(ctx, hipGetLastError());
  }
  return TN_OK;
}

__device__ inline double block_sum256(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

__device__ inline double block_max256(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// sign rule on column j of an n x n matrix in LDS: the first entry within a
// relative 1e-8 of the column's largest magnitude is made positive; returns
// the factor (+1 or -1), identical in every thread
__device__ double column_sign(const double* X, int n, int j, double* red) {
  double mx = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) mx = fmax(mx, fabs(X[i * n + j]));
  mx = block_max256(mx, red);
  // the first qualifying row: smallest index, as a max over -index
  double first = -1e30;
  for (int i = threadIdx.x; i < n; i += 256)
    if (fabs(X[i * n + j]) >= (1.0 - 1e-8) * mx) first = fmax(first, -(double)i);
  first = block_max256(first, red);
  const int fi = (int)(-first);
  return (fi >= 0 && fi < n && X[fi * n + j] < 0.0) ? -1.0 : 1.0;
}

// ---------------------------------------------------------------------------
// canonical form (Sec. IV A)
// ---------------------------------------------------------------------------

// M_b = F1^T diag(lam_b) F2 with F = W sqrt(s) (s below CUT * s_max dropped);
// W, S hold the factorisations of V1 (jobs 0..nl-1) and V2 (nl..2nl-1)
__global__ __launch_bounds__(256) void canon_m_kernel(int nl, int n, const double* __restrict__ W,
                                                      const double* __restrict__ S,
                                                      const double* __restrict__ lam,
                                                      double* __restrict__ M) {
  const int b = blockIdx.x;
  const double* W1 = W + (long long)b * n * n;
  const double* W2 = W + (long long)(nl + b) * n * n;
  const double* S1 = S + (long long)b * n;
  const double* S2 = S + (long long)(nl + b) * n;
  const double* lb = lam + (long long)b * n;
  for (int e = threadIdx.x; e < n * n; e += 256) {
    const int k = e / n, m = e % n;
    const double s1 = S1[k] > CUT * S1[0] ? sqrt(S1[k]) : 0.0;
    const double s2 = S2[m] > CUT * S2[0] ? sqrt(S2[m]) : 0.0;
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc += W1[i * n + k] * lb[i] * W2[i * n + m];
    M[(long long)b * n * n + e] = acc * s1 * s2;
  }
}

// Per link: r = W1 S1^-1/2 U, l = V^T S2^-1/2 W2^T (sign rule on the columns
// of r, rows of l flipping with them); lam <- s / |s|; TR <- TR r, TL <- l TL,
// each rescaled to unit Frobenius norm; dl[b] = max |lam_new - lam_old|.
__global__ __launch_bounds__(256) void canon_update_kernel(
    int nl, int n, const double* __restrict__ W, const double* __restrict__ S,
    const double* __restrict__ Um, const double* __restrict__ Sm, const double* __restrict__ Vm,
    double* __restrict__ lam, double* __restrict__ TR, double* __restrict__ TL,
    double* __restrict__ Rout, double* __restrict__ Lout, double* __restrict__ dl) {
  const int b = blockIdx.x;
  __shared__ double r[MAXN * MAXN], l[MAXN * MAXN], red[4];
  const double* W1 = W + (long long)b * n * n;
  const double* W2 = W + (long long)(nl + b) * n * n;
  const double* S1 = S + (long long)b * n;
  const double* S2 = S + (long long)(nl + b) * n;
  const double* U = Um + (long long)b * n * n;
  const double* V = Vm + (long long)b * n * n;
  const long long nn = (long long)n * n;
  for (int e = threadIdx.x; e < n * n; e += 256) {
    const int i = e / n, j = e % n;
    double a = 0.0, c = 0.0;
    for (int k = 0; k < n; ++k) {
      const double i1 = S1[k] > CUT * S1[0] ? 1.0 / sqrt(S1[k]) : 0.0;
      const double i2 = S2[k] > CUT * S2[0] ? 1.0 / sqrt(S2[k]) : 0.0;
      a += W1[i * n + k] * i1 * U[k * n + j];
      // l[i][j] = sum_k V[k][i] i2_k W2[j][k]
      c += V[k * n + i] * i2 * W2[j * n + k];
    }
    r[e] = a;
    l[e] = c;
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double sg = column_sign(r, n, j, red);
    if (sg < 0.0) {
      for (int i = threadIdx.x; i < n; i += 256) {
        r[i * n + j] = -r[i * n + j];
        l[j * n + i] = -l[j * n + i];
      }
    }
    __syncthreads();
  }
  // spectrum
  double ss = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) ss += Sm[(long long)b * n + i] * Sm[(long long)b * n + i];
  const double snorm = sqrt(block_sum256(ss, red));
  double dmax = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double v = Sm[(long long)b * n + i] / snorm;
    dmax = fmax(dmax, fabs(v - lam[(long long)b * n + i]));
    lam[(long long)b * n + i] = v;
  }
  dmax = block_max256(dmax, red);
  if (threadIdx.x == 0) dl[b] = dmax;
  for (int e = threadIdx.x; e < n * n; e += 256) {
    Rout[b * nn + e] = r[e];
    Lout[b * nn + e] = l[e];
  }
  // TR <- TR r, TL <- l TL (in registers: each thread owns up to 4 entries)
  double nr[EPT], nlv[EPT];
  double s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = threadIdx.x + q * 256;
    nr[q] = nlv[q] = 0.0;
    if (e < n * n) {
      const int i = e / n, j = e % n;
      double a = 0.0, c = 0.0;
      for (int k = 0; k < n; ++k) {
        a += TR[b * nn + i * n + k] * r[k * n + j];
        c += l[i * n + k] * TL[b * nn + k * n + j];
      }
      nr[q] = a;
      nlv[q] = c;
      s1 += a * a;
      s2 += c * c;
    }
  }
  const double n1 = sqrt(block_sum256(s1, red));
  const double n2 = sqrt(block_sum256(s2, red));
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = threadIdx.x + q * 256;
    if (e < n * n) {
      TR[b * nn + e] = nr[q] / n1;
      TL[b * nn + e] = nlv[q] / n2;
    }
  }
}

__global__ void max_of_kernel(const double* __restrict__ x, int n, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double m = 0.0;
  for (int i = 0; i < n; ++i) m = fmax(m, x[i]);
  *out = m;
}

__global__ void eye_kernel(double* __restrict__ X, int batch, int n) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)batch * n * n) return;
  const int e = (int)(t % ((long long)n * n));
  X[t] = (e / n == e % n) ? 1.0 : 0.0;
}

__global__ void fill_kernel(double* __restrict__ X, long long n, double v) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) X[t] = v;
}

// Pc = TR diag(sqrt lam), Qc = diag(sqrt lam) TL per link (one block each),
// then the sign rule on the columns of Pc with the rows of Qc flipping along
// and the scale fixed by |Pc|_F = |Qc|_F: the canonical gauge is unique up
// to these signs and scale, so this makes it independent of the path of the
// iteration
__global__ __launch_bounds__(256) void canon_pq_kernel(int n, const double* __restrict__ TR,
                                                       const double* __restrict__ TL,
                                                       const double* __restrict__ lam,
                                                       double* __restrict__ Pc,
                                                       double* __restrict__ Qc) {
  const int b = blockIdx.x;
  const long long nn = (long long)n * n;
  __shared__ double p[MAXN * MAXN], red[4];
  for (int e = threadIdx.x; e < n * n; e += 256) {
    const int i = e / n, j = e % n;
    p[e] = TR[b * nn + e] * sqrt(lam[(long long)b * n + j]);
    Qc[b * nn + e] = sqrt(lam[(long long)b * n + i]) * TL[b * nn + e];
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double sg = column_sign(p, n, j, red);
    if (sg < 0.0)
      for (int i = threadIdx.x; i < n; i += 256) {
        p[i * n + j] = -p[i * n + j];
        Qc[b * nn + (long long)j * n + i] = -Qc[b * nn + (long long)j * n + i];
      }
    __syncthreads();
  }
  // the scale is free as well: Pc and Qc are inverse up to a factor, and
  // Pc -> c Pc, Qc -> Qc / c is removed by the site normalisation; fix
  // Pc Qc = I (through its trace) and |Pc|_F = |Qc|_F
  double np2 = 0.0, nq2 = 0.0, tr = 0.0;
  for (int e = threadIdx.x; e < n * n; e += 256) {
    const int i = e / n, j = e % n;
    np2 += p[e] * p[e];
    nq2 += Qc[b * nn + e] * Qc[b * nn + e];
    tr += p[e] * Qc[b * nn + (long long)j * n + i];
  }
  np2 = block_sum256(np2, red);
  nq2 = block_sum256(nq2, red);
  tr = block_sum256(tr, red);
  const double m = sqrt((double)n / tr);
  const double r = sqrt(sqrt(nq2) / sqrt(np2));
  for (int e = threadIdx.x; e < n * n; e += 256) {
    Pc[b * nn + e] = p[e] * m * r;
    Qc[b * nn + e] *= m / r;
  }
}

// ---------------------------------------------------------------------------
// gauge fixing (Sec. IV B)
// ---------------------------------------------------------------------------

// U = W V^T per matrix (the orthogonal polar factor of K = W S V^T)
__global__ void polar_kernel(int n, const double* __restrict__ W, const double* __restrict__ V,
                             double* __restrict__ U) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int i = e / n, j = e % n;
  double a = 0.0;
  for (int k = 0; k < n; ++k) a += W[i * n + k] * V[j * n + k];
  U[e] = a;
}

__global__ __launch_bounds__(1024) void dot_kernel(const double* __restrict__ a,
                                                   const double* __restrict__ b, long long n,
                                                   double* __restrict__ out) {
  __shared__ double part[16];
  double s = 0.0;
  for (long long i = threadIdx.x; i < n; i += 1024) s += a[i] * b[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += part[w];
    *out = t;
  }
}

// ---------------------------------------------------------------------------
// gates (Sec. VI A, Fig. 20)
// ---------------------------------------------------------------------------

// iPEPO of the TFIM, g[l][r][d][u][s][s'] = g_F (R_l L_r L_d R_u) g_F with the
// interaction exp(dt J sz sz) = sum_k L_k (x) R_k, L = {sqrt(cosh) I,
// sqrt|sinh| sz}, R = {sqrt(cosh) I, sign(sinh) sqrt|sinh| sz}, and the half
// field step g_F = exp(dt h sx / 2); the left (top) site of a bond takes L on
// its r (d) leg, the right (bottom) site R on its l (u) leg.
void tfim_ipepo(double J, double h, double dt, double* g) {
  const double c = cosh(0.5 * dt * h), s = sinh(0.5 * dt * h);
  const double gf[2][2] = {{c, s}, {s, c}};
  const double ch = cosh(dt * J), sh = sinh(dt * J);
  const double lw[2] = {sqrt(ch), sqrt(fabs(sh))};
  const double rw[2] = {sqrt(ch), (sh < 0 ? -1.0 : 1.0) * sqrt(fabs(sh))};
  for (int l = 0; l < 2; ++l)
    for (int r = 0; r < 2; ++r)
      for (int d = 0; d < 2; ++d)
        for (int u = 0; u < 2; ++u) {
          double mid[2];
          for (int q = 0; q < 2; ++q) {
            const double z = q == 0 ? 1.0 : -1.0;
            const int zp = l + r + d + u;  // total power of sz on this diagonal
            double w = rw[l] * lw[r] * lw[d] * rw[u];
            mid[q] = w * ((zp & 1) ? z : 1.0);
          }
          for (int s1 = 0; s1 < 2; ++s1)
            for (int t1 = 0; t1 < 2; ++t1) {
              double acc = 0.0;
              for (int q = 0; q < 2; ++q) acc += gf[s1][q] * mid[q] * gf[q][t1];
              g[((((l * 2 + r) * 2 + d) * 2 + u) * 2 + s1) * 2 + t1] = acc;
            }
        }
}

// Theta[s][(l,a)][(r,b)][(d,c)][(u,e)] = sum_t g[a][b][c][e][s][t] A[t][l][r][d][u]
__global__ void ipepo_apply_kernel(const double* __restrict__ g, const double* __restrict__ A,
                                   double* __restrict__ Th, int d, int D) {
  const int K = 2, DK = D * K;
  const long long tot = (long long)d * DK * DK * DK * DK;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= tot) return;
  long long r = t;
  const int ue = (int)(r % DK); r /= DK;
  const int dc = (int)(r % DK); r /= DK;
  const int rb = (int)(r % DK); r /= DK;
  const int la = (int)(r % DK); r /= DK;
  const int s = (int)r;
  const int l = la / K, a = la % K, rr = rb / K, b = rb % K, dd = dc / K, c = dc % K, u = ue / K,
            e = ue % K;
  const long long D4 = (long long)D * D * D * D;
  const long long off = (((long long)l * D + rr) * D + dd) * D + u;
  double acc = 0.0;
  for (int tt = 0; tt < d; ++tt)
    acc += g[((((a * K + b) * K + c) * K + e) * d + s) * d + tt] * A[tt * D4 + off];
  Th[t] = acc;
}

// ---------------------------------------------------------------------------
// bond environment (Sec. VI B) and ALS (Eqs. (var), (var1))
// ---------------------------------------------------------------------------

struct Env {
  int chi, D;
  const double* C;
  const double* T;
  const double* Cp(int p, int k) const { return C + ((long long)p * 4 + (k & 3)) * chi * chi; }
  const double* Tp(int p, int k) const {
    return T + ((long long)p * 4 + (k & 3)) * (long long)chi * D * D * chi;
  }
};

// Ns = (N + N^T) / 2 for N an m x m matrix
__global__ void symmetrize_kernel(const double* __restrict__ N, double* __restrict__ Ns, int m) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)m * m) return;
  const int i = (int)(t / m), j = (int)(t % m);
  Ns[t] = 0.5 * (N[t] + N[(long long)j * m + i]);
}

// tb[i][j] = sum_a N[i][j][a][a]; t = <I|N|I> = sum_{i,a} N[i][i][a][a]
__global__ __launch_bounds__(256) void als_traces_kernel(const double* __restrict__ N, int n,
                                                         double* __restrict__ tb,
                                                         double* __restrict__ tconst) {
  __shared__ double red[4];
  const long long n2 = (long long)n * n;
  double t = 0.0;
  for (int e = threadIdx.x; e < n * n; e += 256) {
    double a = 0.0;
    for (int q = 0; q < n; ++q) a += N[(long long)e * n2 + q * n + q];
    tb[e] = a;
    if (e / n == e % n) t += a;
  }
  t = block_sum256(t, red);
  if (threadIdx.x == 0) *tconst = t;
}

// Normal equations of one ALS half step (Eq. (var1)), symmetrised:
// mode 0 (P given Q):  R[(i c),(i' c')] = sum_{j j'} Q[c,j] N[i,j,i',j'] Q[c',j'],
//                      S[(i c)] = sum_j Q[c,j] tb[i,j]
// mode 1 (Q given P):  R[(c j),(c' j')] = sum_{i i'} P[i,c] N[i,j,i',j'] P[i',c'],
//                      S[(c j)] = sum_i P[i,c] tb[i,j]
// F is Q (D x n) for mode 0 and P (n x D) for mode 1.
__global__ void als_normal_kernel(int mode, const double* __restrict__ N,
                                  const double* __restrict__ tb, const double* __restrict__ F,
                                  int n, int D, double* __restrict__ R, double* __restrict__ S) {
  const int k = n * D;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)k * k + k) return;
  const long long n2 = (long long)n * n, n3 = n2 * n;
  if (t >= (long long)k * k) {
    const int row = (int)(t - (long long)k * k);
    double a = 0.0;
    if (mode == 0) {
      const int i = row / D, c = row % D;
      for (int j = 0; j < n; ++j) a += F[c * n + j] * tb[i * n + j];
    } else {
      const int c = row / n, j = row % n;
      for (int i = 0; i < n; ++i) a += F[i * D + c] * tb[i * n + j];
    }
    S[row] = a;
    return;
  }
  const int r1 = (int)(t / k), r2 = (int)(t % k);
  double a = 0.0, b = 0.0;
  if (mode == 0) {
    const int i = r1 / D, c = r1 % D, ip = r2 / D, cp = r2 % D;
    for (int j = 0; j < n; ++j)
      for (int jp = 0; jp < n; ++jp) {
        const double q = F[c * n + j] * F[cp * n + jp];
        a += q * N[i * n3 + j * n2 + ip * n + jp];
        b += q * N[ip * n3 + jp * n2 + i * n + j];
      }
  } else {
    const int c = r1 / n, j = r1 % n, cp = r2 / n, jp = r2 % n;
    for (int i = 0; i < n; ++i)
      for (int ip = 0; ip < n; ++ip) {
        const double q = F[i * D + c] * F[ip * D + cp];
        a += q * N[i * n3 + j * n2 + ip * n + jp];
        b += q * N[ip * n3 + jp * n2 + i * n + j];
      }
  }
  R[t] = 0.5 * (a + b);
}

// x = (R + shift I)^-1 S with shift = shift_rel tr(R), by Gaussian
// elimination with partial pivoting (the first row of largest magnitude) in
// LDS, one workgroup.  R is symmetric but need not be positive definite: with
// an environment N that is not positive, the ALS normal matrix is indefinite.
// info = 0, or j + 1 when pivot j is zero.
__global__ __launch_bounds__(1024) void lu_solve_kernel(int k, const double* __restrict__ R,
                                                        double shift_rel,
                                                        const double* __restrict__ S,
                                                        double* __restrict__ x,
                                                        int* __restrict__ info) {
  extern __shared__ double lds[];
  const int ld = k + 1;                // row stride of the augmented matrix [A | S]
  double* M = lds;                     // k x (k + 1)
  __shared__ double shift;
  __shared__ int piv, fail;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid < 64) {
    double tr = 0.0;
    for (int i = tid; i < k; i += 64) tr += R[(long long)i * k + i];
    for (int o = 32; o > 0; o >>= 1) tr += __shfl_xor(tr, o, 64);
    if (tid == 0) {
      shift = shift_rel * tr;
      fail = 0;
    }
  }
  __syncthreads();
  for (int t = tid; t < k * ld; t += nt) {
    const int i = t / ld, j = t % ld;
    M[t] = j < k ? R[(long long)i * k + j] + (i == j ? shift : 0.0) : S[i];
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    if (tid < 64) {  // pivot: the first row of largest magnitude in column j
      double best = -1.0;
      int bi = k;
      for (int i = j + tid; i < k; i += 64) {
        const double a = fabs(M[i * ld + j]);
        if (a > best) {
          best = a;
          bi = i;
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (tid == 0) {
        piv = bi;
        if (!(best > 0.0) && !fail) fail = j + 1;
      }
    }
    __syncthreads();
    if (fail) break;
    const int p = piv;
    if (p != j)
      for (int c = j + tid; c < ld; c += nt) {
        const double t = M[j * ld + c];
        M[j * ld + c] = M[p * ld + c];
        M[p * ld + c] = t;
      }
    __syncthreads();
    const double inv = 1.0 / M[j * ld + j];
    const int w = ld - j - 1;  // columns right of j, including S
    for (int t = tid; t < (k - j - 1) * w; t += nt) {
      const int i = j + 1 + t / w, c = j + 1 + t % w;
      M[i * ld + c] -= M[i * ld + j] * inv * M[j * ld + c];
    }
    __syncthreads();
  }
  if (tid == 0) *info = fail;
  if (fail) return;
  // back substitution, one column at a time
  for (int j = k - 1; j >= 0; --j) {
    const double xj = M[j * ld + k] / M[j * ld + j];
    for (int i = tid; i < j; i += nt) M[i * ld + k] -= M[i * ld + j] * xj;
    if (tid == 0) x[j] = xj;
    __syncthreads();
  }
}

// O = P Q (n x n)
__global__ void pq_kernel(int n, int D, const double* __restrict__ P, const double* __restrict__ Q,
                          double* __restrict__ O) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int i = e / n, j = e % n;
  double a = 0.0;
  for (int c = 0; c < D; ++c) a += P[i * D + c] * Q[c * n + j];
  O[e] = a;
}

// balance: P = u[:, :D] sqrt(s), Q = sqrt(s) V[:, :D]^T
__global__ void als_balance_kernel(int n, int D, const double* __restrict__ u,
                                   const double* __restrict__ s, const double* __restrict__ V,
                                   double* __restrict__ P, double* __restrict__ Q) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * D) return;
  const int i = e / D, c = e % D;
  const double sq = sqrt(s[c]);
  P[i * D + c] = u[i * n + c] * sq;
  Q[c * n + i] = sq * V[i * n + c];
}

// P[b] = mean of Pz[s] over the slots s that hold link b (Q likewise); a
// link held by one slot takes its truncation as it is
__global__ void slot_mean_kernel(int nl, int per, int l0, int l1, int l2, int l3,
                                 const double* __restrict__ Pz, const double* __restrict__ Qz,
                                 double* __restrict__ P, double* __restrict__ Q) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nl * per) return;
  const int b = (int)(t / per), e = (int)(t % per);
  const int sl[4] = {l0, l1, l2, l3};
  double p = 0.0, q = 0.0;
  int cnt = 0;
  for (int s = 0; s < 4; ++s)
    if (sl[s] == b) {
      p += Pz[(long long)s * per + e];
      q += Qz[(long long)s * per + e];
      ++cnt;
    }
  if (cnt) {
    P[t] = p / cnt;
    Q[t] = q / cnt;
  }
}

// f = t - 2 <PQ|N|I> + <PQ|N|PQ> (Eq. (var), real case); out[0] = f
__global__ __launch_bounds__(256) void als_cost_kernel(int n, int D, const double* __restrict__ N,
                                                       const double* __restrict__ tb,
                                                       const double* __restrict__ tconst,
                                                       const double* __restrict__ P,
                                                       const double* __restrict__ Q,
                                                       double* __restrict__ out) {
  __shared__ double O[MAXN * MAXN], red[4];
  const int n2 = n * n;
  for (int e = threadIdx.x; e < n2; e += 256) {
    const int i = e / n, j = e % n;
    double a = 0.0;
    for (int c = 0; c < D; ++c) a += P[i * D + c] * Q[c * n + j];
    O[e] = a;
  }
  __syncthreads();
  double c = 0.0, q = 0.0;
  for (int e = threadIdx.x; e < n2; e += 256) {
    c += O[e] * tb[e];
    double row = 0.0;
    for (int f = 0; f < n2; ++f) row += N[(long long)e * n2 + f] * O[f];
    q += O[e] * row;
  }
  c = block_sum256(c, red);
  q = block_sum256(q, red);
  if (threadIdx.x == 0) out[0] = tconst[0] - 2.0 * c + q;
}

// Rf = P Pc U (Dk x D), Lf = U^T Qc Q (D x Dk), one link per block row
__global__ void renorm_gate_kernel(int nl, int Dk, int D, const double* __restrict__ P,
                                   const double* __restrict__ Q, const double* __restrict__ Pc,
                                   const double* __restrict__ Qc, const double* __restrict__ U,
                                   double* __restrict__ Rf, double* __restrict__ Lf) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long per = (long long)Dk * D;
  if (t >= 2 * nl * per) return;
  const int which = (int)(t / (nl * per));
  const long long r = t % (nl * per);
  const int b = (int)(r / per);
  const int e = (int)(r % per);
  const double* Pb = P + b * per;
  const double* Qb = Q + b * per;
  const double* Pcb = Pc + (long long)b * D * D;
  const double* Qcb = Qc + (long long)b * D * D;
  const double* Ub = U + (long long)b * D * D;
  if (which == 0) {
    // Rf[i][j] = sum_{a,c} P[i][a] Pc[a][c] U[c][j]
    const int i = e / D, j = e % D;
    double acc = 0.0;
    for (int a = 0; a < D; ++a) {
      double pu = 0.0;
      for (int c = 0; c < D; ++c) pu += Pcb[a * D + c] * Ub[c * D + j];
      acc += Pb[i * D + a] * pu;
    }
    Rf[b * per + e] = acc;
  } else {
    // Lf[j][i] = sum_{a,c} U[a][j] Qc[a][c] Q[c][i]
    const int j = e / Dk, i = e % Dk;
    double acc = 0.0;
    for (int c = 0; c < D; ++c) {
      double uq = 0.0;
      for (int a = 0; a < D; ++a) uq += Ub[a * D + j] * Qcb[a * D + c];
      acc += uq * Qb[c * Dk + i];
    }
    Lf[b * per + e] = acc;
  }
}

// E = mean over positions of -J <zz>_h - J <zz>_v - h <x> (Sec. VI A)
__global__ void tfim2d_energy_kernel(int npos, const double* __restrict__ rho1,
                                     const double* __restrict__ rhoh,
                                     const double* __restrict__ rhov, double J, double h,
                                     double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double zz[4] = {1.0, -1.0, -1.0, 1.0};
  double e = 0.0;
  for (int p = 0; p < npos; ++p) {
    double ch = 0.0, cv = 0.0;
    for (int k = 0; k < 4; ++k) {
      ch += zz[k] * rhoh[p * 16 + k * 4 + k];
      cv += zz[k] * rhov[p * 16 + k * 4 + k];
    }
    const double x = rho1[p * 4 + 1] + rho1[p * 4 + 2];
    e += -J * ch - J * cv - h * x;
  }
  *out = e / npos;
}

inline unsigned nblk(long long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

int check_bond(tn_ctx* ctx, int n, const char* what) {
  if (n < 1 || n > MAXN) TN_FAIL(ctx, TN_EINVAL, "%s = %d outside [1, %d]", what, n, MAXN);
  return TN_OK;
}

BondNet net_of_cell(const CellLinks& L, int nsite, int d) {
  BondNet net;
  net.nsite = nsite;
  net.nl = L.nl;
  net.link.assign(nsite, {-1, -1, -1, -1, -1});
  net.ext.assign(nsite, {d, 0, 0, 0, 0});
  for (int s = 0; s < nsite; ++s)
    for (int ax = 1; ax <= 4; ++ax) net.link[s][ax] = L.leg_link[s][ax];
  for (int b = 0; b < L.nl; ++b) {
    net.s1.push_back(L.s1[b]);
    net.a1.push_back(L.l1[b]);
    net.s2.push_back(L.s2[b]);
    net.a2.push_back(L.l2[b]);
  }
  return net;
}

TDims net_dims(const BondNet& net, int s, int n) {
  TDims t;
  for (int k = 0; k < 5; ++k) t.n[k] = net.link[s][k] >= 0 ? n : net.ext[s][k];
  return t;
}

long long net_max_size(const BondNet& net, int n) {
  long long m = 0;
  for (int s = 0; s < net.nsite; ++s) m = std::max(m, net.size(s, n));
  return m;
}

}  // namespace

// ---------------------------------------------------------------------------
// network-level canonical form, truncation and gauge fixing
// ---------------------------------------------------------------------------

int canonical_pq(tn_ctx* ctx, int nl, int n, const double* P, const double* Q, double* Pc,
                 double* Qc) {
  if (n < 1 || n > MAXN) TN_FAIL(ctx, TN_EINVAL, "canonical gauge needs 1 <= n <= %d", MAXN);
  const size_t mark = ctx->arena_off;  // consumed in stream order
  double* ones = ws_alloc<double>(ctx, (size_t)nl * n);
  if (!ones) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted (canonical gauge)");
  hipLaunchKernelGGL(fill_kernel, dim3(nblk(nl * n)), dim3(256), 0, ctx->stream, ones,
                     (long long)nl * n, 1.0);
  hipLaunchKernelGGL(canon_pq_kernel, dim3(nl), dim3(256), 0, ctx->stream, n, P, Q, ones, Pc, Qc);
  TN_HIP(ctx, hipGetLastError());
  ctx->arena_off = mark;
  return TN_OK;
}

BondNet bondnet_chain2(int d) {
  BondNet net;
  net.nsite = 2;
  net.nl = 2;
  net.link = {{1, -1, 0, -1, -1}, {0, -1, 1, -1, -1}};
  net.ext = {{0, d, 0, 1, 1}, {0, d, 0, 1, 1}};
  net.s1 = {0, 1};
  net.a1 = {2, 2};
  net.s2 = {1, 0};
  net.a2 = {0, 0};
  return net;
}

size_t bondnet_canon_bytes(const BondNet& net, int n) {
  const size_t tsz = (size_t)net_max_size(net, n), nl = net.nl, nn = (size_t)n * n;
  size_t b = 0;
  auto add = [&](size_t c) { b += ((c * 8 + 255) / 256) * 256; };
  add(net.nsite * tsz);  // gammas
  add(tsz);              // ping-pong
  add(2 * tsz);          // apply scratch
  add(nl * n);           // lam
  for (int k = 0; k < 4; ++k) add(nl * nn);  // TR TL R L
  add(2 * nl * nn);                          // grams
  add(2 * nl * nn + 2 * nl * n);             // W S
  add(3 * nl * nn + nl * n);                 // M, Um, Vm, Sm
  add(nl + 1);
  return b + (1 << 16);
}

size_t bondnet_gauge_bytes(const BondNet& net, int n) {
  const size_t tsz = (size_t)net_max_size(net, n), nn = (size_t)n * n;
  size_t b = 0;
  auto add = [&](size_t c) { b += ((c * 8 + 255) / 256) * 256; };
  add(2 * tsz);
  add(2 * tsz);
  add(tsz);
  for (int k = 0; k < 3; ++k) add(nn);
  add(n);
  add(2 * net.nsite + 2);
  return b + (1 << 16);
}

int bondnet_truncate(tn_ctx* ctx, const BondNet& net, int n_in, int n_out, const double* in,
                     const double* P, const double* Q, double* out, double* sc) {
  const long long per = (long long)n_in * n_out;
  long long oin = 0, oout = 0;
  const long long tmax = net_max_size(net, n_in);
  for (int s = 0; s < net.nsite; ++s) {
    LegMats lm;
    for (int ax = 0; ax <= 4; ++ax) {
      const int b = net.link[s][ax];
      if (b < 0) continue;
      const bool first = net.first_end(s, ax);
      lm.m[ax] = (first ? P : Q) + b * per;
      lm.trans[ax] = first ? 1 : 0;
      lm.nnew[ax] = n_out;
    }
    TN_TRY(apply_legs(ctx, in + oin, out + oout, net_dims(net, s, n_in), lm, sc, sc + tmax,
                      nullptr));
    TN_TRY(frob_normalize(ctx, out + oout, net.size(s, n_out), nullptr));
    oin += net.size(s, n_in);
    oout += net.size(s, n_out);
  }
  return TN_OK;
}

int bondnet_canonicalize(tn_ctx* ctx, const BondNet& net, int n, const double* A, double tol,
                         int max_iter, double* lams, double* Pc, double* Qc, double* Aout,
                         int* iters) {
  const int nl = net.nl, nsite = net.nsite;
  const long long tmax = net_max_size(net, n);
  const long long nn = (long long)n * n;
  std::vector<long long> off(nsite + 1, 0);
  for (int s = 0; s < nsite; ++s) off[s + 1] = off[s] + net.size(s, n);
  double* gam = ws_alloc<double>(ctx, off[nsite]);
  double* pp = ws_alloc<double>(ctx, tmax);
  double* sc = ws_alloc<double>(ctx, 2 * tmax);
  double* lam = ws_alloc<double>(ctx, nl * n);
  double* TR = ws_alloc<double>(ctx, nl * nn);
  double* TL = ws_alloc<double>(ctx, nl * nn);
  double* Rm = ws_alloc<double>(ctx, nl * nn);
  double* Lm = ws_alloc<double>(ctx, nl * nn);
  double* G = ws_alloc<double>(ctx, 2 * nl * nn);
  double* W = ws_alloc<double>(ctx, 2 * nl * nn);
  double* S = ws_alloc<double>(ctx, 2 * nl * n);
  double* M = ws_alloc<double>(ctx, nl * nn);
  double* Um = ws_alloc<double>(ctx, nl * nn);
  double* Vm = ws_alloc<double>(ctx, nl * nn);
  double* Sm = ws_alloc<double>(ctx, nl * n);
  double* dl = ws_alloc<double>(ctx, nl + 1);
  if (!dl) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted (canonical form)");
  TN_HIP(ctx, hipMemcpyAsync(gam, A, off[nsite] * sizeof(double), hipMemcpyDeviceToDevice,
                             ctx->stream));
  hipLaunchKernelGGL(fill_kernel, dim3(nblk(nl * n)), dim3(256), 0, ctx->stream, lam,
                     (long long)nl * n, 1.0 / sqrt((double)n));
  hipLaunchKernelGGL(eye_kernel, dim3(nblk(nl * nn)), dim3(256), 0, ctx->stream, TR, nl, n);
  hipLaunchKernelGGL(eye_kernel, dim3(nblk(nl * nn)), dim3(256), 0, ctx->stream, TL, nl, n);
  TN_HIP(ctx, hipGetLastError());
  int it = 0;
  double delta = INFINITY;
  for (it = 1; it <= max_iter; ++it) {
    // Gram matrices of the weighted gammas on each end of each link
    std::vector<GramJob> jobs;
    for (int side = 0; side < 2; ++side)
      for (int b = 0; b < nl; ++b) {
        const int s = side ? net.s2[b] : net.s1[b];
        const int ax = side ? net.a2[b] : net.a1[b];
        GramJob j;
        std::memset(&j, 0, sizeof(j));
        j.A[0] = j.B[0] = gam + off[s];
        j.nterm = 1;
        j.dims = net_dims(net, s, n);
        j.ax[0] = ax;
        for (int k = 0; k < 5; ++k)
          j.lam[k] = (k == ax || net.link[s][k] < 0) ? nullptr
                                                       : lam + (long long)net.link[s][k] * n;
        j.out = G + (side * nl + b) * nn;
        jobs.push_back(j);
      }
    TN_TRY(run_grams(ctx, jobs));
    TN_TRY(jacobi_svd(ctx, 2 * nl, n, n, G, n, nn, W, n, nn, S, n, nullptr, 0, 0));
    hipLaunchKernelGGL(canon_m_kernel, dim3(nl), dim3(256), 0, ctx->stream, nl, n, W, S, lam, M);
    TN_TRY(jacobi_svd(ctx, nl, n, n, M, n, nn, Um, n, nn, Sm, n, Vm, n, nn));
    hipLaunchKernelGGL(canon_update_kernel, dim3(nl), dim3(256), 0, ctx->stream, nl, n, W, S, Um,
                       Sm, Vm, lam, TR, TL, Rm, Lm, dl);
    TN_HIP(ctx, hipGetLastError());
    // gammas: first end new = r^T old, second end new = l old
    for (int s = 0; s < nsite; ++s) {
      LegMats lm;
      for (int ax = 0; ax <= 4; ++ax) {
        const int b = net.link[s][ax];
        if (b < 0) continue;
        const bool first = net.first_end(s, ax);
        lm.m[ax] = (first ? Rm : Lm) + b * nn;
        lm.trans[ax] = first ? 1 : 0;
        lm.nnew[ax] = n;
      }
      const long long ts = net.size(s, n);
      TN_TRY(apply_legs(ctx, gam + off[s], pp, net_dims(net, s, n), lm, sc, sc + tmax, nullptr));
      TN_HIP(ctx, hipMemcpyAsync(gam + off[s], pp, ts * sizeof(double), hipMemcpyDeviceToDevice,
                                 ctx->stream));
      TN_TRY(frob_normalize(ctx, gam + off[s], ts, nullptr));
    }
    hipLaunchKernelGGL(max_of_kernel, dim3(1), dim3(1), 0, ctx->stream, dl, nl, dl + nl);
    TN_HIP(ctx, hipMemcpyAsync(ctx->host_scratch, dl + nl, sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
    delta = ctx->host_scratch[0];
    if (!std::isfinite(delta)) TN_FAIL(ctx, TN_ENUMERIC, "non-finite canonical-form spectra");
    if (delta < tol) break;
  }
  hipLaunchKernelGGL(canon_pq_kernel, dim3(nl), dim3(256), 0, ctx->stream, n, TR, TL, lam, Pc, Qc);
  TN_HIP(ctx, hipGetLastError());
  if (lams)
    TN_HIP(ctx, hipMemcpyAsync(lams, lam, (size_t)nl * n * sizeof(double), hipMemcpyDeviceToDevice,
                               ctx->stream));
  if (Aout) TN_TRY(bondnet_truncate(ctx, net, n, n, A, Pc, Qc, Aout, sc));
  if (iters) *iters = std::min(it, max_iter);
  return delta < tol ? TN_OK : TN_NOT_CONVERGED;
}

int bondnet_gauge_fix(tn_ctx* ctx, const BondNet& net, int n, const double* a_ref,
                      const double* a_new, double* U, double tol, int max_iter, double* fidelity,
                      int* iters) {
  const int nl = net.nl, nsite = net.nsite;
  if (nsite > 30) TN_FAIL(ctx, TN_EINVAL, "gauge fixing handles at most 30 site tensors");
  const long long tmax = net_max_size(net, n), nn = (long long)n * n;
  std::vector<long long> off(nsite + 1, 0);
  for (int s = 0; s < nsite; ++s) off[s + 1] = off[s] + net.size(s, n);
  double* rest = ws_alloc<double>(ctx, 2 * tmax);
  double* sc = ws_alloc<double>(ctx, 2 * tmax);
  double* full = ws_alloc<double>(ctx, tmax);
  double* K = ws_alloc<double>(ctx, nn);
  double* Wk = ws_alloc<double>(ctx, nn);
  double* Vk = ws_alloc<double>(ctx, nn);
  double* Sk = ws_alloc<double>(ctx, n);
  double* dots = ws_alloc<double>(ctx, 2 * nsite + 2);
  if (!dots) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted (gauge fix)");
  // norms of both sets (fixed)
  for (int s = 0; s < nsite; ++s) {
    const long long ts = net.size(s, n);
    hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(1024), 0, ctx->stream, a_ref + off[s],
                       a_ref + off[s], ts, dots + nsite + s);
    hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(1024), 0, ctx->stream, a_new + off[s],
                       a_new + off[s], ts, dots + s);
  }
  TN_HIP(ctx, hipMemcpyAsync(ctx->host_scratch, dots, 2 * nsite * sizeof(double),
                             hipMemcpyDeviceToHost, ctx->stream));
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  double den = 0.0;
  for (int s = 0; s < nsite; ++s)
    den += sqrt(ctx->host_scratch[s]) * sqrt(ctx->host_scratch[nsite + s]);
  if (!(den > 0.0)) TN_FAIL(ctx, TN_EINVAL, "zero site tensor");
  // U applied as new = U old on every link leg (optionally all but one)
  auto legs_of = [&](int s, int skip) {
    LegMats lm;
    for (int ax = 0; ax <= 4; ++ax) {
      const int b = net.link[s][ax];
      if (b < 0 || ax == skip) continue;
      lm.m[ax] = U + b * nn;
      lm.nnew[ax] = n;
    }
    return lm;
  };
  auto fid = [&](double* F) -> int {
    for (int s = 0; s < nsite; ++s) {
      TN_TRY(apply_legs(ctx, a_ref + off[s], full, net_dims(net, s, n), legs_of(s, -1), sc,
                        sc + tmax, nullptr));
      hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(1024), 0, ctx->stream, a_new + off[s], full,
                         net.size(s, n), dots + s);
    }
    TN_HIP(ctx, hipMemcpyAsync(ctx->host_scratch, dots, nsite * sizeof(double),
                               hipMemcpyDeviceToHost, ctx->stream));
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
    double num = 0.0;
    for (int s = 0; s < nsite; ++s) num += ctx->host_scratch[s];
    *F = num / den;
    return TN_OK;
  };
  double F = 0.0;
  TN_TRY(fid(&F));
  int it = 0;
  double dF = INFINITY;
  for (it = 1; it <= max_iter; ++it) {
    // one Procrustes step per link, the other links' factors held fixed
    for (int b = 0; b < nl; ++b) {
      GramJob j;
      std::memset(&j, 0, sizeof(j));
      j.nterm = 2;
      j.out = K;
      for (int side = 0; side < 2; ++side) {
        const int s = side ? net.s2[b] : net.s1[b];
        const int leg = side ? net.a2[b] : net.a1[b];
        TN_TRY(apply_legs(ctx, a_ref + off[s], rest + side * tmax, net_dims(net, s, n),
                          legs_of(s, leg), sc, sc + tmax, nullptr));
        j.A[side] = a_new + off[s];
        j.B[side] = rest + side * tmax;
        j.ax[side] = leg;
        j.dims = net_dims(net, s, n);
      }
      if (net.size(net.s1[b], n) != net.size(net.s2[b], n))
        TN_FAIL(ctx, TN_EINVAL, "internal: link ends of different tensor sizes");
      TN_TRY(run_grams(ctx, {j}));
      TN_TRY(jacobi_svd(ctx, 1, n, n, K, n, nn, Wk, n, nn, Sk, n, Vk, n, nn));
      hipLaunchKernelGGL(polar_kernel, dim3(nblk(nn)), dim3(256), 0, ctx->stream, n, Wk, Vk,
                         U + b * nn);
      TN_HIP(ctx, hipGetLastError());
    }
    double Fn = 0.0;
    TN_TRY(fid(&Fn));
    if (!std::isfinite(Fn)) TN_FAIL(ctx, TN_ENUMERIC, "non-finite fidelity");
    dF = fabs(Fn - F);
    F = Fn;
    if (dF < tol) break;
  }
  if (fidelity) *fidelity = F;
  if (iters) *iters = std::min(it, max_iter);
  return dF < tol ? TN_OK : TN_NOT_CONVERGED;
}

namespace {

int truncate_sites(tn_ctx* ctx, const CellLinks& L, int nsite, int d, int n_in, int n_out,
                   const double* in, const double* P, const double* Q, double* out, double* sc) {
  return bondnet_truncate(ctx, net_of_cell(L, nsite, d), n_in, n_out, in, P, Q, out, sc);
}

}  // namespace

// ---------------------------------------------------------------------------
// public entry points (C ABI wrappers live in abi.hip)
// ---------------------------------------------------------------------------

int cell_links_impl(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, int* nlink,
                    int* links) {
  CellLinks L;
  TN_TRY(build_links(ctx, Lx, Ly, nsite, cell, L));
  if (nlink) *nlink = L.nl;
  if (links)
    for (int b = 0; b < L.nl; ++b) {
      links[4 * b + 0] = L.s1[b];
      links[4 * b + 1] = L.l1[b];
      links[4 * b + 2] = L.s2[b];
      links[4 * b + 3] = L.l2[b];
    }
  return TN_OK;
}

int ipeps_gate_impl(tn_ctx* ctx, int nsite, int D, int d, double J, double h, double dt,
                    const double* A, double* Theta) {
  if (nsite < 1 || D < 1 || d != 2 || !A || !Theta)
    TN_FAIL(ctx, TN_EINVAL, "ipeps_gate needs nsite >= 1, D >= 1, d = 2 and device tensors");
  TN_TRY(check_bond(ctx, 2 * D, "kappa*D"));
  double hg[64];
  tfim_ipepo(J, h, dt, hg);
  TN_TRY(ws_reserve(ctx, 1 << 16));
  ws_reset(ctx);
  double* g = ws_alloc<double>(ctx, 64);
  if (!g) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted");
  TN_HIP(ctx, hipMemcpyAsync(g, hg, sizeof(hg), hipMemcpyHostToDevice, ctx->stream));
  const long long ain = (long long)d * D * D * D * D;
  const long long aout = ain * 16;
  for (int s = 0; s < nsite; ++s)
    hipLaunchKernelGGL(ipepo_apply_kernel, dim3(nblk(aout)), dim3(256), 0, ctx->stream, g,
                       A + s * ain, Theta + s * aout, d, D);
  TN_HIP(ctx, hipGetLastError());
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return TN_OK;
}

int ipeps_truncate_impl(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, int d, int Din,
                        int Dout, const double* Theta, const double* P, const double* Q,
                        double* Aout) {
  CellLinks L;
  TN_TRY(build_links(ctx, Lx, Ly, nsite, cell, L));
  TN_TRY(check_bond(ctx, Din, "input bond"));
  TN_TRY(check_bond(ctx, Dout, "output bond"));
  if (d < 1 || !Theta || !P || !Q || !Aout) TN_FAIL(ctx, TN_EINVAL, "null tensor argument");
  const long long tin = (long long)d * Din * Din * Din * Din;
  TN_TRY(ws_reserve(ctx, 2 * tin * sizeof(double) + (1 << 20)));
  ws_reset(ctx);
  double* sc = ws_alloc<double>(ctx, 2 * tin);
  if (!sc) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted");
  TN_TRY(truncate_sites(ctx, L, nsite, d, Din, Dout, Theta, P, Q, Aout, sc));
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return TN_OK;
}

int ipeps_canonicalize_impl(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, int d, int D,
                            int Dkeep, const double* A, double* Aout, double* lams, double* P,
                            double* Q, double tol, int max_iter, int* iters) {
  CellLinks L;
  TN_TRY(build_links(ctx, Lx, Ly, nsite, cell, L));
  TN_TRY(check_bond(ctx, D, "bond"));
  if (Dkeep < 1 || Dkeep > D) TN_FAIL(ctx, TN_EINVAL, "kept bond %d outside [1, %d]", Dkeep, D);
  if (d < 1 || !A || !P || !Q) TN_FAIL(ctx, TN_EINVAL, "null tensor argument");
  if (max_iter < 1) TN_FAIL(ctx, TN_EINVAL, "max_iter must be >= 1");
  if (Aout && Dkeep != D) TN_FAIL(ctx, TN_EINVAL, "A_out needs the full bond (Dkeep = D)");
  const BondNet net = net_of_cell(L, nsite, d);
  const int nl = L.nl;
  const long long nn = (long long)D * D;
  TN_TRY(ws_reserve(ctx, bondnet_canon_bytes(net, D) + 2 * nl * nn * sizeof(double) +
                             (1 << 20)));
  ws_reset(ctx);
  double* Pc = ws_alloc<double>(ctx, nl * nn);
  double* Qc = ws_alloc<double>(ctx, nl * nn);
  if (!Qc) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted");
  int it = 0;
  const int rc = bondnet_canonicalize(ctx, net, D, A, tol, max_iter, lams, Pc, Qc, Aout, &it);
  if (rc < 0) return rc;
  // kept columns of Pc and rows of Qc
  TN_HIP(ctx, hipMemcpy2DAsync(P, Dkeep * sizeof(double), Pc, D * sizeof(double),
                               Dkeep * sizeof(double), (size_t)nl * D, hipMemcpyDeviceToDevice,
                               ctx->stream));
  for (int b = 0; b < nl; ++b)
    TN_HIP(ctx, hipMemcpyAsync(Q + (long long)b * Dkeep * D, Qc + b * nn,
                               (size_t)Dkeep * D * sizeof(double), hipMemcpyDeviceToDevice,
                               ctx->stream));
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (iters) *iters = it;
  return rc;
}

int gauge_fix_impl(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, int d, int D,
                   const double* a_ref, const double* a_new, double* U, double tol, int max_iter,
                   double* fidelity, int* iters) {
  CellLinks L;
  TN_TRY(build_links(ctx, Lx, Ly, nsite, cell, L));
  TN_TRY(check_bond(ctx, D, "bond"));
  if (d < 1 || !a_ref || !a_new || !U) TN_FAIL(ctx, TN_EINVAL, "null tensor argument");
  if (max_iter < 1) TN_FAIL(ctx, TN_EINVAL, "max_iter must be >= 1");
  const BondNet net = net_of_cell(L, nsite, d);
  TN_TRY(ws_reserve(ctx, bondnet_gauge_bytes(net, D) + (1 << 20)));
  ws_reset(ctx);
  return bondnet_gauge_fix(ctx, net, D, a_ref, a_new, U, tol, max_iter, fidelity, iters);
}

namespace {

// ---------------------------------------------------------------------------
// the truncation block (Sec. VI B, Fig. 21(a)): a 2x2 block of sites, its
// four internal links (slots) and the CTM environment around it
// ---------------------------------------------------------------------------

// block positions (x, y) = (0, 0), (1, 0), (1, 1), (0, 1)
enum { B_TL = 0, B_TR = 1, B_BR = 2, B_BL = 3 };
// slots in visiting order: top, left, bottom, right; the first end carries P
struct SlotDef {
  int e1, ax1, e2, ax2;
};
constexpr SlotDef SLOT[4] = {{B_TL, AX_R, B_TR, AX_L},
                             {B_TL, AX_D, B_BL, AX_U},
                             {B_BL, AX_R, B_BR, AX_L},
                             {B_TR, AX_D, B_BR, AX_U}};

// slot of axis ax of block position X, or -1 when the axis faces the environment
int slot_of(int X, int ax) {
  for (int k = 0; k < 4; ++k) {
    if (SLOT[k].e1 == X && SLOT[k].ax1 == ax) return k;
    if (SLOT[k].e2 == X && SLOT[k].ax2 == ax) return k;
  }
  return -1;
}

// How the internal links of a layer are closed: truncated by the slots'
// current (P, Q), or left at the full bond (the gated state Psi_g).
enum { L_ZETA = 0, L_FULL = 1 };

struct Block {
  const CellLinks* L;
  int d, D, n, chi;  // D: the slots' truncated bond, n: the full bond kappa D
  int pos[4], site[4], slot_link[4];
  Env env;
  const double* Theta;  // [nsite][d][n]^4
  const double *Psu, *Qsu;  // [nlink][n][De], [nlink][De][n]: legs facing the environment
  double *Pz, *Qz;          // [4][n][D], [4][D][n]: the slots' current truncation
  size_t big;               // doubles of the largest corner or ring intermediate
  double *ket[4], *bra[4], *sc1, *sc2;
  TDims kd[4], bd[4];
  double *E[4], *X1, *X2, *X3, *R1, *R2;
  int De = 0;  // bond of the legs facing the environment (the environment's bond)

  static size_t big_of(int d, int De, int n, int chi) {
    const size_t c2 = (size_t)chi * chi, n2 = (size_t)n * n;
    return std::max(c2 * n2 * n2, c2 * (size_t)De * De * d * n2);
  }
  static size_t bytes(int d, int D, int De, int n, int chi) {
    const size_t tsz = (size_t)d * n * n * n * n, big = big_of(d, De, n, chi);
    size_t need = 0;
    auto add = [&](size_t c) { need += ((c * 8 + 255) / 256) * 256; };
    for (int k = 0; k < 8; ++k) add(tsz);   // ket, bra per position
    add(tsz);
    add(tsz);                                // apply_legs scratch
    for (int k = 0; k < 4; ++k) add(big);    // corners
    add((size_t)chi * chi * De * De);        // X1
    add(big);                                // X2 (chi^2 D^4 fits)
    add(big);                                // X3
    add(big);
    add(big);                                // ring intermediates
    add(4 * (size_t)n * D);
    add(4 * (size_t)n * D);                  // Pz, Qz
    return need;
  }

  int alloc(tn_ctx* ctx) {
    const size_t tsz = (size_t)d * n * n * n * n;
    big = big_of(d, De, n, chi);
    for (int k = 0; k < 4; ++k) {
      ket[k] = ws_alloc<double>(ctx, tsz);
      bra[k] = ws_alloc<double>(ctx, tsz);
    }
    sc1 = ws_alloc<double>(ctx, tsz);
    sc2 = ws_alloc<double>(ctx, tsz);
    for (int k = 0; k < 4; ++k) E[k] = ws_alloc<double>(ctx, big);
    X1 = ws_alloc<double>(ctx, (size_t)chi * chi * De * De);
    X2 = ws_alloc<double>(ctx, big);
    X3 = ws_alloc<double>(ctx, big);
    R1 = ws_alloc<double>(ctx, big);
    R2 = ws_alloc<double>(ctx, big);
    Pz = ws_alloc<double>(ctx, 4 * (size_t)n * D);
    Qz = ws_alloc<double>(ctx, 4 * (size_t)n * D);
    if (!Qz) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted (truncation block)");
    return TN_OK;
  }

  // Site tensor of block position X for one layer: legs facing the
  // environment truncated by the pre-truncation, internal legs by the
  // slot's (Pz, Qz) (mode L_ZETA, except the open slot) or untruncated.
  int layer(tn_ctx* ctx, int X, int mode, int open, double* out, TDims* dout) {
    const int s = site[X];
    LegMats lm;
    for (int ax = 1; ax <= 4; ++ax) {
      const int k = slot_of(X, ax);
      if (k < 0) {
        const int b = L->leg_link[s][ax];
        const bool first = (L->s1[b] == s && L->l1[b] == ax);
        lm.m[ax] = (first ? Psu : Qsu) + (long long)b * n * De;
        lm.trans[ax] = first ? 1 : 0;
        lm.nnew[ax] = De;
      } else if (k != open && mode == L_ZETA) {
        const bool first = SLOT[k].e1 == X;
        lm.m[ax] = (first ? Pz : Qz) + (long long)k * n * D;
        lm.trans[ax] = first ? 1 : 0;
        lm.nnew[ax] = D;
      }
    }
    return apply_legs(ctx, Theta + (long long)s * d * n * n * n * n, out, dims5(d, n, n, n, n),
                      lm, sc1, sc2, dout);
  }

  // The four enlarged corners of the block, ket and bra layers as given:
  //   E_TL[t, rk, rb, dk, db, x], E_TR[t, lk, lb, dk, db, f],
  //   E_BR[f, uk, ub, lk, lb, y], E_BL[y, rk, rb, uk, ub, x]
  int corners(tn_ctx* ctx, int kmode, int bmode, int open) {
    for (int X = 0; X < 4; ++X) {
      TN_TRY(layer(ctx, X, kmode, open, ket[X], &kd[X]));
      TN_TRY(layer(ctx, X, bmode, open, bra[X], &bd[X]));
    }
    const int c = chi, e = De, dd = d;
    auto K = [&](int X, int ax) { return kd[X].n[ax]; };
    auto Bd = [&](int X, int ax) { return bd[X].n[ax]; };
    // top-left: C1 of TL, T1 of TL, T4 of TL
    {
      const int X = B_TL, p = pos[X];
      TN_TRY(ein(ctx, "xlLg,gh->xlLh", env.Tp(p, 3), {c, e, e, c}, env.Cp(p, 0), {c, c}, X1));
      TN_TRY(ein(ctx, "xlLh,huUt->xlLuUt", X1, {c, e, e, c}, env.Tp(p, 0), {c, e, e, c}, X2));
      TN_TRY(ein(ctx, "xlLuUt,slrdu->xLUtsrd", X2, {c, e, e, e, e, c}, ket[X],
                 {dd, e, K(X, AX_R), K(X, AX_D), e}, X3));
      TN_TRY(ein(ctx, "xLUtsrd,sLRDU->trRdDx", X3, {c, e, e, c, dd, K(X, AX_R), K(X, AX_D)},
                 bra[X], {dd, e, Bd(X, AX_R), Bd(X, AX_D), e}, E[X]));
    }
    // top-right: T1 of TR, C2 of TR, T2 of TR
    {
      const int X = B_TR, p = pos[X];
      TN_TRY(ein(ctx, "tuUh,he->tuUe", env.Tp(p, 0), {c, e, e, c}, env.Cp(p, 1), {c, c}, X1));
      TN_TRY(ein(ctx, "tuUe,erRf->tuUrRf", X1, {c, e, e, c}, env.Tp(p, 1), {c, e, e, c}, X2));
      TN_TRY(ein(ctx, "tuUrRf,slrdu->tURfsld", X2, {c, e, e, e, e, c}, ket[X],
                 {dd, K(X, AX_L), e, K(X, AX_D), e}, X3));
      TN_TRY(ein(ctx, "tURfsld,sLRDU->tlLdDf", X3, {c, e, e, c, dd, K(X, AX_L), K(X, AX_D)},
                 bra[X], {dd, Bd(X, AX_L), e, Bd(X, AX_D), e}, E[X]));
    }
    // bottom-right: T2 of BR, C3 of BR, T3 of BR
    {
      const int X = B_BR, p = pos[X];
      TN_TRY(ein(ctx, "frRg,gh->frRh", env.Tp(p, 1), {c, e, e, c}, env.Cp(p, 2), {c, c}, X1));
      TN_TRY(ein(ctx, "frRh,hdDy->frRdDy", X1, {c, e, e, c}, env.Tp(p, 2), {c, e, e, c}, X2));
      TN_TRY(ein(ctx, "frRdDy,slrdu->fRDysul", X2, {c, e, e, e, e, c}, ket[X],
                 {dd, K(X, AX_L), e, e, K(X, AX_U)}, X3));
      TN_TRY(ein(ctx, "fRDysul,sLRDU->fuUlLy", X3, {c, e, e, c, dd, K(X, AX_U), K(X, AX_L)},
                 bra[X], {dd, Bd(X, AX_L), e, e, Bd(X, AX_U)}, E[X]));
    }
    // bottom-left: T3 of BL, C4 of BL, T4 of BL
    {
      const int X = B_BL, p = pos[X];
      TN_TRY(ein(ctx, "ydDg,ge->ydDe", env.Tp(p, 2), {c, e, e, c}, env.Cp(p, 3), {c, c}, X1));
      TN_TRY(ein(ctx, "ydDe,elLx->ydDlLx", X1, {c, e, e, c}, env.Tp(p, 3), {c, e, e, c}, X2));
      TN_TRY(ein(ctx, "ydDlLx,slrdu->yDLxsru", X2, {c, e, e, e, e, c}, ket[X],
                 {dd, e, K(X, AX_R), e, K(X, AX_U)}, X3));
      TN_TRY(ein(ctx, "yDLxsru,sLRDU->yrRuUx", X3, {c, e, e, c, dd, K(X, AX_R), K(X, AX_U)},
                 bra[X], {dd, e, Bd(X, AX_R), e, Bd(X, AX_U)}, E[X]));
    }
    return TN_OK;
  }

  // The ring with slot `open` cut, scaled by alpha: out[i][j][i'][j'], i, j
  // the ket index of the slot's first and second end, i', j' the bra index;
  // open < 0 closes every link and writes the scalar norm network.
  int ring(tn_ctx* ctx, int open, double alpha, double* out) {
    const int c = chi;
    const std::initializer_list<int> tl = {c, kd[0].n[AX_R], bd[0].n[AX_R], kd[0].n[AX_D],
                                           bd[0].n[AX_D], c};
    const std::initializer_list<int> tr = {c, kd[1].n[AX_L], bd[1].n[AX_L], kd[1].n[AX_D],
                                           bd[1].n[AX_D], c};
    const std::initializer_list<int> br = {c, kd[2].n[AX_U], bd[2].n[AX_U], kd[2].n[AX_L],
                                           bd[2].n[AX_L], c};
    const std::initializer_list<int> bl = {c, kd[3].n[AX_R], bd[3].n[AX_R], kd[3].n[AX_U],
                                           bd[3].n[AX_U], c};
    const int a = kd[0].n[AX_R], A = bd[0].n[AX_R], b = kd[0].n[AX_D], B = bd[0].n[AX_D];
    const int e = kd[1].n[AX_D], Ee = bd[1].n[AX_D], h = kd[2].n[AX_L], H = bd[2].n[AX_L];
    switch (open) {
      case 0:  // top
        TN_TRY(ein(ctx, "feEhHy,yhHbBx->feEbBx", E[2], br, E[3], bl, R1));
        TN_TRY(ein(ctx, "taAbBx,feEbBx->taAfeE", E[0], tl, R1, {c, e, Ee, b, B, c}, R2));
        TN_TRY(ein(ctx, "taAfeE,tcCeEf->acAC", R2, {c, a, A, c, e, Ee}, E[1], tr, out, alpha));
        break;
      case 1:  // left
        TN_TRY(ein(ctx, "taAeEf,feEhHy->taAhHy", E[1], tr, E[2], br, R1));
        TN_TRY(ein(ctx, "taAbBx,taAhHy->bBxhHy", E[0], tl, R1, {c, a, A, h, H, c}, R2));
        TN_TRY(ein(ctx, "bBxhHy,yhHmMx->bmBM", R2, {b, B, c, h, H, c}, E[3], bl, out, alpha));
        break;
      case 2:  // bottom
        TN_TRY(ein(ctx, "taAbBx,taAeEf->bBxeEf", E[0], tl, E[1], tr, R1));
        TN_TRY(ein(ctx, "bBxeEf,feEhHy->bBxhHy", R1, {b, B, c, e, Ee, c}, E[2], br, R2));
        TN_TRY(ein(ctx, "bBxhHy,ykKbBx->khKH", R2, {b, B, c, h, H, c}, E[3], bl, out, alpha));
        break;
      case 3:  // right
        TN_TRY(ein(ctx, "yhHbBx,taAbBx->yhHtaA", E[3], bl, E[0], tl, R1));
        TN_TRY(ein(ctx, "yhHtaA,taAeEf->yhHeEf", R1, {c, h, H, c, a, A}, E[1], tr, R2));
        TN_TRY(ein(ctx, "yhHeEf,fgGhHy->egEG", R2, {c, h, H, e, Ee, c}, E[2], br, out, alpha));
        break;
      default:  // closed
        TN_TRY(ein(ctx, "taAbBx,taAeEf->bBxeEf", E[0], tl, E[1], tr, R1));
        TN_TRY(ein(ctx, "bBxeEf,feEhHy->bBxhHy", R1, {b, B, c, e, Ee, c}, E[2], br, R2));
        TN_TRY(ein(ctx, "bBxhHy,yhHbBx->", R2, {b, B, c, h, H, c}, E[3], bl, out, alpha));
    }
    return TN_OK;
  }

  // The two environments of slot k (raw ring sign times sg): N with zeta in
  // both layers, symmetrised in ket <-> bra (Ns), and M with zeta in the ket
  // layer against the untruncated bra layer of Psi_g.
  int envs(tn_ctx* ctx, int k, double sg, double* N, double* Ns, double* M) {
    TN_TRY(corners(ctx, L_ZETA, L_ZETA, k));
    TN_TRY(ring(ctx, k, sg, N));
    const long long n2 = (long long)n * n;
    hipLaunchKernelGGL(symmetrize_kernel, dim3(nblk(n2 * n2)), dim3(256), 0, ctx->stream, N, Ns,
                       (int)n2);
    TN_HIP(ctx, hipGetLastError());
    TN_TRY(corners(ctx, L_ZETA, L_FULL, k));
    return ring(ctx, k, sg, M);
  }
};

// Block geometry of a cell: positions, sites and the cell link of each slot;
// TN_EINVAL when the block at the origin does not hold every link.
int block_setup(tn_ctx* ctx, const CellLinks& L, int Lx, int Ly, const int* cell, Block& B) {
  auto pos = [&](int x, int y) { return (y % Ly) * Lx + (x % Lx); };
  B.pos[B_TL] = pos(0, 0);
  B.pos[B_TR] = pos(1, 0);
  B.pos[B_BR] = pos(1, 1);
  B.pos[B_BL] = pos(0, 1);
  for (int X = 0; X < 4; ++X) B.site[X] = cell[B.pos[X]];
  bool seen[MAXL] = {false};
  for (int k = 0; k < 4; ++k) {
    const int s1 = B.site[SLOT[k].e1], s2 = B.site[SLOT[k].e2];
    const int b = L.leg_link[s1][SLOT[k].ax1];
    if (b < 0 || L.leg_link[s2][SLOT[k].ax2] != b || L.s1[b] != s1 || L.s2[b] != s2)
      TN_FAIL(ctx, TN_EINVAL, "internal: slot %d does not match the cell links", k);
    B.slot_link[k] = b;
    seen[b] = true;
  }
  for (int b = 0; b < L.nl; ++b)
    if (!seen[b])
      TN_FAIL(ctx, TN_EINVAL, "link %d of the cell lies outside the 2x2 truncation block", b);
  return TN_OK;
}

int bond_env_check(tn_ctx* ctx, int d, int D, int Dk, int De, int chi, const void* Theta,
                   const void* C, const void* T, const void* Psu, const void* Qsu) {
  TN_TRY(check_bond(ctx, Dk, "theta bond"));
  if (D < 1 || D > Dk) TN_FAIL(ctx, TN_EINVAL, "truncated bond %d outside [1, %d]", D, Dk);
  if (De < 1 || De > Dk)
    TN_FAIL(ctx, TN_EINVAL, "environment bond %d outside [1, %d]", De, Dk);
  if (d < 1 || chi < 1 || !Theta || !C || !T || !Psu || !Qsu)
    TN_FAIL(ctx, TN_EINVAL, "bad bond environment arguments");
  const double big = (double)Block::big_of(d, De, Dk, chi);
  if (big > 2.0e9) TN_FAIL(ctx, TN_EINVAL, "truncation block too large (chi %d, bond %d)", chi, Dk);
  return TN_OK;
}

}  // namespace

int bond_environment_impl(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, int d, int D,
                          int Dk, int De, const double* Theta, int chi, const double* C,
                          const double* T, const double* Psu, const double* Qsu,
                          const double* P, const double* Q,
                          int slot, double* N_out, double* M_out) {
  CellLinks L;
  TN_TRY(build_links(ctx, Lx, Ly, nsite, cell, L));
  TN_TRY(bond_env_check(ctx, d, D, Dk, De, chi, Theta, C, T, Psu, Qsu));
  if (!P || !Q) TN_FAIL(ctx, TN_EINVAL, "null truncation");
  if (slot < 0 || slot > 3) TN_FAIL(ctx, TN_EINVAL, "slot %d outside [0, 4)", slot);
  if (!N_out || !M_out) TN_FAIL(ctx, TN_EINVAL, "null output");
  const size_t n4 = (size_t)Dk * Dk * Dk * Dk;
  TN_TRY(ws_reserve(ctx, Block::bytes(d, D, De, Dk, chi) + n4 * 8 + (1 << 20)));
  ws_reset(ctx);
  Block B{&L, d, D, Dk, chi, {}, {}, {}, Env{chi, De, C, T}, Theta, Psu, Qsu};
  B.De = De;
  TN_TRY(block_setup(ctx, L, Lx, Ly, cell, B));
  TN_TRY(B.alloc(ctx));
  double* Nraw = ws_alloc<double>(ctx, n4);
  if (!Nraw) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted (bond environment)");
  const size_t per = (size_t)Dk * D;
  for (int k = 0; k < 4; ++k) {
    TN_HIP(ctx, hipMemcpyAsync(B.Pz + k * per, P + B.slot_link[k] * per, per * 8,
                               hipMemcpyDeviceToDevice, ctx->stream));
    TN_HIP(ctx, hipMemcpyAsync(B.Qz + k * per, Q + B.slot_link[k] * per, per * 8,
                               hipMemcpyDeviceToDevice, ctx->stream));
  }
  TN_TRY(B.envs(ctx, slot, 1.0, Nraw, N_out, M_out));
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return TN_OK;
}

int bond_env_truncate_impl(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, int d, int D,
                           int Dk, int De, const double* Theta, int chi, const double* C,
                           const double* T, const double* Psu, const double* Qsu,
                           double* P, double* Q,
                           int max_passes, int max_sweeps, double tol, double* cost, int* passes,
                           int* sweeps) {
  CellLinks L;
  TN_TRY(build_links(ctx, Lx, Ly, nsite, cell, L));
  TN_TRY(bond_env_check(ctx, d, D, Dk, De, chi, Theta, C, T, Psu, Qsu));
  if (!P || !Q) TN_FAIL(ctx, TN_EINVAL, "null truncation");
  if (max_passes < 1 || max_sweeps < 1)
    TN_FAIL(ctx, TN_EINVAL, "max_passes and max_sweeps must be >= 1");
  const int n = Dk, k = Dk * D;
  // the augmented k x (k + 1) system of the solve lives in LDS
  if (k > 140) TN_FAIL(ctx, TN_EINVAL, "kappa*D*D = %d too large for the ALS solve", k);
  const size_t n_ = n, n4 = n_ * n_ * n_ * n_;
  size_t need = Block::bytes(d, D, De, Dk, chi);
  auto add = [&](size_t c) { need += ((c * 8 + 255) / 256) * 256; };
  add(3 * n4);                          // N raw, N symmetrised, M
  add(n_ * n_ + 4);                     // tb, T, scratch
  add(4 * (size_t)k * k + 2 * k);       // R and S
  add(4 * n_ * n_ + n_ + 8);            // O, u, V, s, f
  add(64);                              // info
  TN_TRY(ws_reserve(ctx, need + (1 << 20)));
  ws_reset(ctx);
  Block B{&L, d, D, Dk, chi, {}, {}, {}, Env{chi, De, C, T}, Theta, Psu, Qsu};
  B.De = De;
  TN_TRY(block_setup(ctx, L, Lx, Ly, cell, B));
  TN_TRY(B.alloc(ctx));
  double* Nraw = ws_alloc<double>(ctx, 3 * n4);
  double* Ns = Nraw + n4;
  double* M = Ns + n4;
  double* tb = ws_alloc<double>(ctx, n_ * n_ + 4);
  double* tdev = tb + n_ * n_;          // <Psi_g|Psi_g>
  double* tjunk = tdev + 1;
  double* R = ws_alloc<double>(ctx, 4 * (size_t)k * k + 2 * k);
  double* S = R + 4 * (size_t)k * k;
  double* O = ws_alloc<double>(ctx, 4 * n_ * n_ + n_ + 8);
  double* uo = O + n_ * n_;
  double* Vo = uo + n_ * n_;
  double* so = Vo + n_ * n_;
  double* fdev = so + n_;
  int* info = ws_alloc<int>(ctx, 64);
  if (!info) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted (ALS)");
  const size_t per = (size_t)Dk * D;
  for (int s = 0; s < 4; ++s) {
    TN_HIP(ctx, hipMemcpyAsync(B.Pz + s * per, P + B.slot_link[s] * per, per * 8,
                               hipMemcpyDeviceToDevice, ctx->stream));
    TN_HIP(ctx, hipMemcpyAsync(B.Qz + s * per, Q + B.slot_link[s] * per, per * 8,
                               hipMemcpyDeviceToDevice, ctx->stream));
  }
  // <Psi_g|Psi_g>: the closed block with every internal link untruncated; the
  // normalised boundary leaves the common sign of all networks free, take
  // the one that makes it positive
  TN_TRY(B.corners(ctx, L_FULL, L_FULL, -1));
  TN_TRY(B.ring(ctx, -1, 1.0, tdev));
  TN_HIP(ctx, hipMemcpyAsync(ctx->host_scratch, tdev, sizeof(double), hipMemcpyDeviceToHost,
                             ctx->stream));
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  const double traw = ctx->host_scratch[0];
  if (!std::isfinite(traw) || traw == 0.0)
    TN_FAIL(ctx, TN_ENUMERIC, "block norm %g is not a usable scale", traw);
  const double sg = traw > 0 ? 1.0 : -1.0, tn = fabs(traw);
  ctx->host_scratch[0] = tn;
  TN_HIP(ctx, hipMemcpyAsync(tdev, ctx->host_scratch, sizeof(double), hipMemcpyHostToDevice,
                             ctx->stream));
  int total_sweeps = 0, pass = 0;
  double f = 0.0, f_prev = 0.0;
  bool have_prev = false;
  for (pass = 1; pass <= max_passes; ++pass) {
    for (int s = 0; s < 4; ++s) {
      TN_TRY(B.envs(ctx, s, sg, Nraw, Ns, M));
      hipLaunchKernelGGL(als_traces_kernel, dim3(1), dim3(256), 0, ctx->stream, M, n, tb, tjunk);
      double* Pb = B.Pz + s * per;
      double* Qb = B.Qz + s * per;
      if (!have_prev) {
        hipLaunchKernelGGL(als_cost_kernel, dim3(1), dim3(256), 0, ctx->stream, n, D, Ns, tb,
                           tdev, Pb, Qb, fdev);
        TN_HIP(ctx, hipGetLastError());
        TN_HIP(ctx, hipMemcpyAsync(ctx->host_scratch, fdev, sizeof(double),
                                   hipMemcpyDeviceToHost, ctx->stream));
        TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
        f_prev = f = ctx->host_scratch[0];
        have_prev = true;
        if (!std::isfinite(f)) TN_FAIL(ctx, TN_ENUMERIC, "non-finite bond environment");
      }
      double fs = f;
      for (int sw = 1; sw <= max_sweeps; ++sw) {
        ++total_sweeps;
        for (int mode = 0; mode < 2; ++mode) {
          hipLaunchKernelGGL(als_normal_kernel, dim3(nblk((long long)k * k + k)), dim3(256), 0,
                             ctx->stream, mode, Ns, tb, mode == 0 ? Qb : Pb, n, D, R, S);
          TN_HIP(ctx, hipGetLastError());
          hipLaunchKernelGGL(lu_solve_kernel, dim3(1), dim3(1024),
                             (size_t)k * (k + 1) * sizeof(double), ctx->stream, k, R, 1e-14, S,
                             mode == 0 ? Pb : Qb, info + mode);
          TN_HIP(ctx, hipGetLastError());
        }
        // balance the pair through the SVD of P Q (P Q, hence f, unchanged)
        hipLaunchKernelGGL(pq_kernel, dim3(nblk((long long)n * n)), dim3(256), 0, ctx->stream, n,
                           D, Pb, Qb, O);
        TN_TRY(jacobi_svd(ctx, 1, n, n, O, n, (long long)n * n, uo, n, (long long)n * n, so, n,
                          Vo, n, (long long)n * n));
        hipLaunchKernelGGL(als_balance_kernel, dim3(nblk((long long)per)), dim3(256), 0,
                           ctx->stream, n, D, uo, so, Vo, Pb, Qb);
        hipLaunchKernelGGL(als_cost_kernel, dim3(1), dim3(256), 0, ctx->stream, n, D, Ns, tb,
                           tdev, Pb, Qb, fdev);
        TN_HIP(ctx, hipGetLastError());
        TN_HIP(ctx, hipMemcpyAsync(ctx->host_scratch, fdev, sizeof(double),
                                   hipMemcpyDeviceToHost, ctx->stream));
        TN_HIP(ctx, hipMemcpyAsync(ctx->host_scratch + 2, info, 2 * sizeof(int),
                                   hipMemcpyDeviceToHost, ctx->stream));
        TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
        const int* hinfo = reinterpret_cast<const int*>(ctx->host_scratch + 2);
        if (hinfo[0] || hinfo[1])
          TN_FAIL(ctx, TN_ENUMERIC, "ALS normal matrix of slot %d singular (pivot %d/%d)", s,
                  hinfo[0], hinfo[1]);
        const double fn = ctx->host_scratch[0];
        if (!std::isfinite(fn)) TN_FAIL(ctx, TN_ENUMERIC, "non-finite ALS cost");
        const bool done = fabs(fn - fs) < tol * tn;
        fs = fn;
        if (done) break;
      }
      f = fs;
    }
    const bool done = fabs(f - f_prev) < tol * tn;
    f_prev = f;
    if (done) break;
  }
  if (pass > max_passes) pass = max_passes;
  // the links' truncations: the mean over the slots that hold each link
  hipLaunchKernelGGL(slot_mean_kernel, dim3(nblk((long long)L.nl * per)), dim3(256), 0,
                     ctx->stream, L.nl, (int)per, B.slot_link[0], B.slot_link[1],
                     B.slot_link[2], B.slot_link[3], B.Pz, B.Qz, P, Q);
  TN_HIP(ctx, hipGetLastError());
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (cost) {
    cost[0] = f;
    cost[1] = tn;
  }
  if (passes) *passes = pass;
  if (sweeps) *sweeps = total_sweeps;
  return TN_OK;
}

int fu_renormalized_gate_impl(tn_ctx* ctx, int nlink, int Dk, int D, const double* P,
                              const double* Q, const double* Pc, const double* Qc, const double* U,
                              double* Rf, double* Lf) {
  if (nlink < 1 || Dk < 1 || D < 1 || D > Dk || !P || !Q || !Pc || !Qc || !U || !Rf || !Lf)
    TN_FAIL(ctx, TN_EINVAL, "bad fu_renormalized_gate arguments");
  TN_TRY(recycle_factors(ctx, nlink, Dk, D, P, Q, Pc, Qc, U, Rf, Lf));
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return TN_OK;
}

int ipeps_energy_impl(tn_ctx* ctx, int Lx, int Ly, int D, int d, int nsite, const double* sites,
                      const int* cell, int chi, const double* C, const double* T, double J,
                      double h, double* energy) {
  if (d != 2) TN_FAIL(ctx, TN_EINVAL, "ipeps_energy is the TFIM energy: d must be 2");
  if (!energy) TN_FAIL(ctx, TN_EINVAL, "null energy pointer");
  if (Lx < 1 || Ly < 1 || Lx * Ly > 64) TN_FAIL(ctx, TN_EINVAL, "bad cell size");
  const int npos = Lx * Ly;
  void* buf = nullptr;
  TN_TRY(keep_buffer(ctx, "energy-rdms", (size_t)(npos * (4 + 16 + 16) + 1) * sizeof(double), &buf,
                     nullptr));
  double* rho1 = static_cast<double*>(buf);
  double* rhoh = rho1 + npos * 4;
  double* rhov = rhoh + npos * 16;
  double* e = rhov + npos * 16;
  TN_TRY(ipeps_rdms_impl(ctx, Lx, Ly, D, d, nsite, sites, cell, chi, C, T, rho1, rhoh, rhov));
  hipLaunchKernelGGL(tfim2d_energy_kernel, dim3(1), dim3(1), 0, ctx->stream, npos, rho1, rhoh,
                     rhov, J, h, e);
  TN_HIP(ctx, hipGetLastError());
  TN_HIP(ctx, hipMemcpyAsync(ctx->host_scratch, e, sizeof(double), hipMemcpyDeviceToHost,
                             ctx->stream));
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *energy = ctx->host_scratch[0];
  if (!std::isfinite(*energy)) TN_FAIL(ctx, TN_ENUMERIC, "non-finite energy");
  return TN_OK;
}

namespace {

// Start of the gauge fix inside the recycling step: for a small time step
// the renormalized gate is close to the identity, so the kappa = 0 block of
// the composite truncation maps the old bond basis onto the new one;
// K = (P Pc)[(i,0), :]^T / |.| + (Qc Q)[:, (i,0)] / |.|, U0 = polar(K).
__global__ __launch_bounds__(256) void gauge_start_kernel(int Dk, int D, int kappa,
                                                          const double* __restrict__ P,
                                                          const double* __restrict__ Q,
                                                          const double* __restrict__ Pc,
                                                          const double* __restrict__ Qc,
                                                          double* __restrict__ K) {
  const int b = blockIdx.x;
  __shared__ double red[4];
  const long long per = (long long)Dk * D, dd = (long long)D * D;
  const double* Pb = P + b * per;
  const double* Qb = Q + b * per;
  const double* Pcb = Pc + b * dd;
  const double* Qcb = Qc + b * dd;
  double a[EPT], c[EPT];
  double na = 0.0, nc = 0.0;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = threadIdx.x + q * 256;
    a[q] = c[q] = 0.0;
    if (e < D * D) {
      const int i = e / D, j = e % D;
      // a = (P Pc)[(j, 0), i]  (transposed block), c = (Qc Q)[i, (j, 0)]
      double x = 0.0, y = 0.0;
      for (int m = 0; m < D; ++m) {
        x += Pb[(long long)(j * kappa) * D + m] * Pcb[m * D + i];
        y += Qcb[i * D + m] * Qb[(long long)m * Dk + j * kappa];
      }
      a[q] = x;
      c[q] = y;
      na += x * x;
      nc += y * y;
    }
  }
  na = sqrt(block_sum256(na, red));
  nc = sqrt(block_sum256(nc, red));
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = threadIdx.x + q * 256;
    if (e < D * D) K[b * dd + e] = a[q] / na + c[q] / nc;
  }
}

}  // namespace

int recycle_gauge_start(tn_ctx* ctx, int nl, int Dk, int D, int kappa, const double* P,
                        const double* Q, const double* Pc, const double* Qc, double* U0) {
  const long long dd = (long long)D * D;
  const size_t mark = ctx->arena_off;
  double* K = ws_alloc<double>(ctx, nl * dd);
  double* W = ws_alloc<double>(ctx, nl * dd);
  double* V = ws_alloc<double>(ctx, nl * dd);
  double* S = ws_alloc<double>(ctx, nl * D);
  if (!S) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted (gauge start)");
  hipLaunchKernelGGL(gauge_start_kernel, dim3(nl), dim3(256), 0, ctx->stream, Dk, D, kappa, P, Q,
                     Pc, Qc, K);
  TN_HIP(ctx, hipGetLastError());
  TN_TRY(jacobi_svd(ctx, nl, D, D, K, D, dd, W, D, dd, S, D, V, D, dd));
  for (int b = 0; b < nl; ++b)
    hipLaunchKernelGGL(polar_kernel, dim3(nblk(dd)), dim3(256), 0, ctx->stream, D, W + b * dd,
                       V + b * dd, U0 + b * dd);
  TN_HIP(ctx, hipGetLastError());
  ctx->arena_off = mark;  // stream order makes the slice reusable
  return TN_OK;
}

int recycle_factors(tn_ctx* ctx, int nl, int Dk, int D, const double* P, const double* Q,
                    const double* Pc, const double* Qc, const double* U, double* Rf, double* Lf) {
  const long long tot = 2LL * nl * Dk * D;
  hipLaunchKernelGGL(renorm_gate_kernel, dim3(nblk(tot)), dim3(256), 0, ctx->stream, nl, Dk, D, P,
                     Q, Pc, Qc, U, Rf, Lf);
  TN_HIP(ctx, hipGetLastError());
  return TN_OK;
}

int fu_gauge_start_impl(tn_ctx* ctx, int nlink, int Dk, int D, int kappa, const double* P,
                        const double* Q, const double* Pc, const double* Qc, double* U0) {
  if (nlink < 1 || D < 1 || kappa < 1 || Dk != kappa * D || !P || !Q || !Pc || !Qc || !U0)
    TN_FAIL(ctx, TN_EINVAL, "bad fu_gauge_start arguments");
  TN_TRY(check_bond(ctx, D, "bond"));
  const long long dd = (long long)D * D;
  TN_TRY(ws_reserve(ctx, (size_t)(4 * nlink * dd + nlink * D) * sizeof(double) + (1 << 20)));
  ws_reset(ctx);
  TN_TRY(recycle_gauge_start(ctx, nlink, Dk, D, kappa, P, Q, Pc, Qc, U0));
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return TN_OK;
}
