// Table-driven tensor contraction on MFMA (FP64 16x16x4 tiles).
//
// A contraction C[m, n] = alpha * sum_k A[m, k] B[k, n] + beta * C[m, n] over
// arbitrary tensor layouts: every operand index group (rows, columns, the
// contracted group) is described by a table of element offsets, so permuted
// operands are read in place and results are written straight into the
// layout the next step needs -- no transpose kernels between contractions.
// Tables are built once per shape on the host and cached in the context.
#include <algorithm>
#include <cstring>
#include <sstream>

#include "common.h"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

struct TDesc {
  int M, N, K;
  const int* am;
  const int* ak;
  const int* bk;
  const int* bn;
  const int* cm;
  const int* cn;
  long long sa, sb, sc;
  int a_mfast, b_nfast;
};

constexpr int BM = 64, BN = 64, BK = 16, PAD = 1;

// 256 threads = 4 waves; each wave owns a 32x32 quarter of the 64x64 tile as
// 2x2 MFMA blocks.  Operand tiles are staged through LDS; the table entries
// of the tile's rows, columns and k-slice are staged too.
__global__ __launch_bounds__(256) void tgemm_f64_kernel(const double* __restrict__ A,
                                                        const double* __restrict__ B,
                                                        double* __restrict__ C, TDesc d,
                                                        double alpha, double beta) {
  __shared__ double As[BK][BM + PAD];
  __shared__ double Bs[BK][BN + PAD];
  __shared__ int sam[BM], sbn[BN], sak[BK], sbk[BK];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const long long bz = blockIdx.z;
  A += bz * d.sa;
  B += bz * d.sb;
  C += bz * d.sc;
  if (tid < BM) {
    sam[tid] = (m0 + tid < d.M) ? d.am[m0 + tid] : 0;
  } else if (tid < BM + BN) {
    const int j = tid - BM;
    sbn[j] = (n0 + j < d.N) ? d.bn[n0 + j] : 0;
  }
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  for (int k0 = 0; k0 < d.K; k0 += BK) {
    __syncthreads();
    if (tid < BK) {
      sak[tid] = (k0 + tid < d.K) ? d.ak[k0 + tid] : 0;
    } else if (tid >= 64 && tid < 64 + BK) {
      const int j = tid - 64;
      sbk[j] = (k0 + j < d.K) ? d.bk[k0 + j] : 0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int m, k;
      if (d.a_mfast) {
        m = tid & 63;
        k = (tid >> 6) + 4 * i;
      } else {
        k = tid & 15;
        m = (tid >> 4) + 16 * i;
      }
      double v = 0.0;
      if (m0 + m < d.M && k0 + k < d.K) v = A[(long long)sam[m] + sak[k]];
      As[k][m] = v;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int n, k;
      if (d.b_nfast) {
        n = tid & 63;
        k = (tid >> 6) + 4 * i;
      } else {
        k = tid & 15;
        n = (tid >> 4) + 16 * i;
      }
      double v = 0.0;
      if (n0 + n < d.N && k0 + k < d.K) v = B[(long long)sbk[k] + sbn[n]];
      Bs[k][n] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kk + (lane >> 4)][wm + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk + (lane >> 4)][wn + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
  // D layout of the 16x16 FP64 block (measured on gfx950): lane l, register r
  // holds row l/16 + 4 r, column l%16
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + (lane >> 4) + 4 * r;
        const int col = n0 + wn + j * 16 + (lane & 15);
        if (row < d.M && col < d.N) {
          const long long off = (long long)d.cm[row] + d.cn[col];
          double v = alpha * acc[i][j][r];
          if (beta != 0.0) v += beta * C[off];
          C[off] = v;
        }
      }
}

std::string key_of(const IdxGroup& g) {
  std::ostringstream s;
  for (size_t i = 0; i < g.ext.size(); ++i) s << g.ext[i] << ':' << g.str[i] << ',';
  return s.str();
}

int table_of(tn_ctx* ctx, const IdxGroup& g, const int** out) {
  const std::string key = key_of(g);
  auto it = ctx->tables.find(key);
  if (it != ctx->tables.end()) {
    *out = it->second;
    return TN_OK;
  }
  const long long n = g.size();
  std::vector<int> h(n > 0 ? n : 1, 0);
  const int nd = (int)g.ext.size();
  std::vector<int> idx(nd, 0);
  for (long long f = 0; f < n; ++f) {
    long long off = 0;
    for (int i = 0; i < nd; ++i) off += idx[i] * g.str[i];
    if (off > 2147483647LL || off < 0)
      TN_FAIL(ctx, TN_EINVAL, "tensor offset %lld exceeds the 32-bit table range", off);
    h[f] = (int)off;
    for (int i = nd - 1; i >= 0; --i) {
      if (++idx[i] < g.ext[i]) break;
      idx[i] = 0;
    }
  }
  int* dptr = nullptr;
  TN_HIP(ctx, hipMalloc(&dptr, h.size() * sizeof(int)));
  TN_HIP(ctx, hipMemcpy(dptr, h.data(), h.size() * sizeof(int), hipMemcpyHostToDevice));
  ctx->tables[key] = dptr;
  *out = dptr;
  return TN_OK;
}

// true when the group's flat index walks memory with unit stride at its fastest end
bool unit_fast(const IdxGroup& g) { return !g.str.empty() && g.str.back() == 1; }

}  // namespace

int tc_run(tn_ctx* ctx, const Contraction& c, const double* A, const double* B, double* C,
           double alpha, double beta, int prec) {
  const long long M = c.am.size(), N = c.bn.size(), K = c.ak.size();
  if (M != c.cm.size() || N != c.cn.size() || K != c.bk.size())
    TN_FAIL(ctx, TN_EINVAL, "contraction groups disagree (M %lld/%lld N %lld/%lld K %lld/%lld)",
            M, c.cm.size(), N, c.cn.size(), K, c.bk.size());
  if (M == 0 || N == 0 || c.batch == 0) return TN_OK;
  if (M > 2147483647LL || N > 65535LL * BN || c.batch > 65535)
    TN_FAIL(ctx, TN_EINVAL, "contraction too large for one launch");
  (void)prec;
  TDesc d;
  d.M = (int)M;
  d.N = (int)N;
  d.K = (int)K;
  TN_TRY(table_of(ctx, c.am, &d.am));
  TN_TRY(table_of(ctx, c.ak, &d.ak));
  TN_TRY(table_of(ctx, c.bk, &d.bk));
  TN_TRY(table_of(ctx, c.bn, &d.bn));
  TN_TRY(table_of(ctx, c.cm, &d.cm));
  TN_TRY(table_of(ctx, c.cn, &d.cn));
  d.sa = c.sa;
  d.sb = c.sb;
  d.sc = c.sc;
  d.a_mfast = unit_fast(c.am) || !unit_fast(c.ak);
  d.b_nfast = unit_fast(c.bn) || !unit_fast(c.bk);
  if (K == 0) {
    // C = beta * C: run with a zero-length k loop
  }
  dim3 grid((unsigned)((M + BM - 1) / BM), (unsigned)((N + BN - 1) / BN), (unsigned)c.batch);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ctx->prof) {
    while (ctx->ev_pool.size() < ctx->ev_used + 2) {
      hipEvent_t e;
      TN_HIP(ctx, hipEventCreate(&e));
      ctx->ev_pool.push_back(e);
    }
    e0 = ctx->ev_pool[ctx->ev_used];
    e1 = ctx->ev_pool[ctx->ev_used + 1];
    ctx->ev_used += 2;
    ctx->prof_flops.push_back(2.0 * (double)M * (double)N * (double)K * (double)c.batch);
    TN_HIP(ctx, hipEventRecord(e0, ctx->stream));
  }
  hipLaunchKernelGGL(tgemm_f64_kernel, grid, dim3(256), 0, ctx->stream, A, B, C, d, alpha, beta);
  TN_HIP(ctx, hipGetLastError());
  if (ctx->prof) TN_HIP(ctx, hipEventRecord(e1, ctx->stream));
  return TN_OK;
}

int gemm(tn_ctx* ctx, int M, int N, int K, const double* A, int lda, bool ta, const double* B,
         int ldb, bool tb, double* C, int ldc, double alpha, double beta, int batch, long long sa,
         long long sb, long long sc, int prec) {
  Contraction c;
  c.am = grp({{M, ta ? 1LL : (long long)lda}});
  c.ak = grp({{K, ta ? (long long)lda : 1LL}});
  c.bk = grp({{K, tb ? 1LL : (long long)ldb}});
  c.bn = grp({{N, tb ? (long long)ldb : 1LL}});
  c.cm = grp({{M, (long long)ldc}});
  c.cn = grp({{N, 1LL}});
  c.batch = batch;
  c.sa = sa;
  c.sb = sb;
  c.sc = sc;
  return tc_run(ctx, c, A, B, C, alpha, beta, prec);
}
