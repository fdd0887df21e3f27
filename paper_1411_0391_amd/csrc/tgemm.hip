// Table-driven tensor contraction on MFMA: FP64 16x16x4 tiles, and the
// reduced-precision bulk forms (FP32 16x16x4 and BF16 16x16x32 with FP32
// accumulation) that read the same FP64 operands, round them while staging
// into LDS and write FP64 results.
//
// A contraction C[m, n] = alpha * sum_k A[m, k] B[k, n] + beta * C[m, n] over
// arbitrary tensor layouts: every operand index group (rows, columns, the
// contracted group) is described by a table of element offsets, so permuted
// operands are read in place and results are written straight into the
// layout the next step needs -- no transpose kernels between contractions.
// Tables are built once per shape on the host and cached in the context.
#include <algorithm>
#include <map>
#include <cstring>
#include <sstream>
#include <type_traits>

#include <hip/hip_ext.h>

#include "common.h"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

struct TDesc {
  int M, N, K;
  // table mode: offset tables; strided mode: element strides
  const int* am;
  const int* ak;
  const int* bk;
  const int* bn;
  const int* cm;
  const int* cn;
  long long sam, sak, sbk, sbn, scm, scn;
  long long sa, sb, sc;  // batch strides
  int a_mfast, b_nfast;
  int ksplit, kchunk;    // split-K: chunk length (multiple of BK)
  double* part;          // split-K partials [batch*ksplit][M][N]
};

constexpr int BM = 64, BN = 64, BK = 16, PAD = 1;

template <bool TABLE>
__device__ inline long long offA(const TDesc& d, int m, int k) {
  if (TABLE) return (long long)d.am[m] + d.ak[k];
  return (long long)m * d.sam + (long long)k * d.sak;
}
template <bool TABLE>
__device__ inline long long offB(const TDesc& d, int k, int n) {
  if (TABLE) return (long long)d.bk[k] + d.bn[n];
  return (long long)k * d.sbk + (long long)n * d.sbn;
}
template <bool TABLE>
__device__ inline long long offC(const TDesc& d, int m, int n) {
  if (TABLE) return (long long)d.cm[m] + d.cn[n];
  return (long long)m * d.scm + (long long)n * d.scn;
}

// 256 threads = 4 waves; the 64 x TBN tile (TBN = 32, 64, 96 or 128) is split
// 2 x 2 between the waves, each owning 32 x TBN/2 as 2 x TBN/32 MFMA blocks.
// The wide tiles serve products with a narrow N (the n x n x k products of
// the projector SVD): the whole width is one tile, so the large operand is
// streamed once.  Operand tiles are staged through two LDS buffers: the
// next k-slice is fetched into registers while the MFMAs consume the current
// one.  With split-K each z-slice of the grid sums one chunk of k into a
// partial tile; a second kernel reduces the partials in a fixed order.
template <bool TABLE, int TBN>
__global__ __launch_bounds__(256) void tgemm_f64_kernel(const double* __restrict__ A,
                                                        const double* __restrict__ B,
                                                        double* __restrict__ C, TDesc d,
                                                        double alpha, double beta) {
  constexpr int NB = TBN * BK / 256;  // B elements a thread stages per slice
  constexpr int NJ = TBN / 32;        // MFMA column blocks per wave
  __shared__ double As[2][BK][BM + PAD];
  __shared__ double Bs[2][BK][TBN + PAD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * TBN;
  const int split = blockIdx.z % d.ksplit;
  const long long bz = blockIdx.z / d.ksplit;
  A += bz * d.sa;
  B += bz * d.sb;
  const int kbeg = split * d.kchunk;
  const int kend = min(d.K, kbeg + d.kchunk);
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * (TBN / 2);
  d4 acc[2][NJ];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  // per-thread coordinates of its 4 A and NB B tile elements
  int am_[4], ak_[4], bk_[NB], bn_[NB];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (d.a_mfast) {
      am_[i] = tid & 63;
      ak_[i] = (tid >> 6) + 4 * i;
    } else {
      ak_[i] = tid & 15;
      am_[i] = (tid >> 4) + 16 * i;
    }
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int e = tid + 256 * i;
    if (d.b_nfast) {
      bn_[i] = e % TBN;
      bk_[i] = e / TBN;
    } else {
      bk_[i] = e % BK;
      bn_[i] = e / BK;
    }
  }
  // The k-independent half of each operand offset, computed once.  Rows of
  // A past M and columns of B past N are clamped into range instead of
  // masked: they only feed outputs that are never stored.  Strided mode
  // folds the element's k within the slice into it as well, so that a full
  // slice's addresses are this plus the slice's uniform k0 offset.
  long long ca[4], cb[NB];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = min(m0 + am_[i], d.M - 1);
    ca[i] = TABLE ? (long long)d.am[m] : (long long)m * d.sam + (long long)ak_[i] * d.sak;
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int n = min(n0 + bn_[i], d.N - 1);
    cb[i] = TABLE ? (long long)d.bn[n] : (long long)n * d.sbn + (long long)bk_[i] * d.sbk;
  }
  double ra[4], rb[NB];
  // a full slice: every k below kend, no tests
  auto fetch = [&](int k0) {
    const double* Ak = TABLE ? A : A + (long long)k0 * d.sak;
    const double* Bk = TABLE ? B : B + (long long)k0 * d.sbk;
#pragma unroll
    for (int i = 0; i < 4; ++i) ra[i] = Ak[TABLE ? ca[i] + d.ak[k0 + ak_[i]] : ca[i]];
#pragma unroll
    for (int i = 0; i < NB; ++i) rb[i] = Bk[TABLE ? cb[i] + d.bk[k0 + bk_[i]] : cb[i]];
  };
  // the ragged last slice: k clamped below kend for the address, the value
  // zeroed past it
  auto fetch_tail = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = min(k0 + ak_[i], kend - 1);
      const double v =
          A[TABLE ? ca[i] + d.ak[k] : ca[i] + (long long)(k - ak_[i]) * d.sak];
      ra[i] = k0 + ak_[i] < kend ? v : 0.0;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int k = min(k0 + bk_[i], kend - 1);
      const double v =
          B[TABLE ? cb[i] + d.bk[k] : cb[i] + (long long)(k - bk_[i]) * d.sbk];
      rb[i] = k0 + bk_[i] < kend ? v : 0.0;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) As[buf][ak_[i]][am_[i]] = ra[i];
#pragma unroll
    for (int i = 0; i < NB; ++i) Bs[buf][bk_[i]][bn_[i]] = rb[i];
  };
  int buf = 0;
  if (kbeg < kend) {
    if (kbeg + BK <= kend) fetch(kbeg); else fetch_tail(kbeg);
    stash(0);
  }
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const int kn = k0 + BK;
    if (kn + BK <= kend) fetch(kn);
    else if (kn < kend) fetch_tail(kn);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double a[2], b[NJ];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[buf][kk + (lane >> 4)][wm + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < NJ; ++j) b[j] = Bs[buf][kk + (lane >> 4)][wn + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (kn < kend) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // D layout of the 16x16 FP64 block (measured on gfx950): lane l, register r
  // holds row l/16 + 4 r, column l%16
  if (d.ksplit == 1) {
    C += bz * d.sc;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm + i * 16 + (lane >> 4) + 4 * r;
          const int col = n0 + wn + j * 16 + (lane & 15);
          if (row < d.M && col < d.N) {
            const long long off = offC<TABLE>(d, row, col);
            double v = alpha * acc[i][j][r];
            if (beta != 0.0) v += beta * C[off];
            C[off] = v;
          }
        }
  } else {
    double* P = d.part + (long long)blockIdx.z * d.M * d.N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm + i * 16 + (lane >> 4) + 4 * r;
          const int col = n0 + wn + j * 16 + (lane & 15);
          if (row < d.M && col < d.N) P[(long long)row * d.N + col] = acc[i][j][r];
        }
  }
}

// Reduced-precision form of the same tiling.  PREC_BF16: operands rounded to
// bf16, k slices of 32 (one 16x16x32 MFMA per 16x16 block and slice), LDS
// tiles k-contiguous so that a lane reads its 8 consecutive k values at once;
// otherwise fp32, k slices of 16 (four 16x16x4 MFMAs).  Accumulation in fp32;
// D layout of both (measured on gfx950): lane l, register r holds row
// 4 (l/16) + r, column l%16.
template <bool BF16, bool TABLE>
__global__ __launch_bounds__(256) void tgemm_lp_kernel(const double* __restrict__ A,
                                                       const double* __restrict__ B,
                                                       double* __restrict__ C, TDesc d,
                                                       double alpha, double beta) {
  constexpr int KB = BF16 ? 32 : 16;
  constexpr int NLD = KB / 4;  // elements of each operand a thread stages per slice
  typedef typename std::conditional<BF16, __bf16, float>::type T;
  // bf16: [row][k] with 8 k of padding (16-byte aligned rows); fp32: [k][row]
  constexpr int R1 = BF16 ? BM : KB, R2 = BF16 ? KB + 8 : BM + PAD;
  __shared__ __attribute__((aligned(16))) T As[2][R1][R2];
  __shared__ __attribute__((aligned(16))) T Bs[2][R1][R2];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int split = blockIdx.z % d.ksplit;
  const long long bz = blockIdx.z / d.ksplit;
  A += bz * d.sa;
  B += bz * d.sb;
  const int kbeg = split * d.kchunk;
  const int kend = min(d.K, kbeg + d.kchunk);
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  int am_[NLD], ak_[NLD], bk_[NLD], bn_[NLD];
#pragma unroll
  for (int i = 0; i < NLD; ++i) {
    if (d.a_mfast) {
      am_[i] = tid & 63;
      ak_[i] = (tid >> 6) + 4 * i;
    } else {
      ak_[i] = tid % KB;
      am_[i] = tid / KB + (256 / KB) * i;
    }
    if (d.b_nfast) {
      bn_[i] = tid & 63;
      bk_[i] = (tid >> 6) + 4 * i;
    } else {
      bk_[i] = tid % KB;
      bn_[i] = tid / KB + (256 / KB) * i;
    }
  }
  double ra[NLD], rb[NLD];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
      const int m = m0 + am_[i], k = k0 + ak_[i];
      ra[i] = (m < d.M && k < kend) ? A[offA<TABLE>(d, m, k)] : 0.0;
      const int n = n0 + bn_[i], kb = k0 + bk_[i];
      rb[i] = (n < d.N && kb < kend) ? B[offB<TABLE>(d, kb, n)] : 0.0;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
      if constexpr (BF16) {
        As[buf][am_[i]][ak_[i]] = (__bf16)(float)ra[i];
        Bs[buf][bn_[i]][bk_[i]] = (__bf16)(float)rb[i];
      } else {
        As[buf][ak_[i]][am_[i]] = (float)ra[i];
        Bs[buf][bk_[i]][bn_[i]] = (float)rb[i];
      }
    }
  };
  int buf = 0;
  if (kbeg < kend) {
    fetch(kbeg);
    stash(0);
  }
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += KB) {
    const bool more = k0 + KB < kend;
    if (more) fetch(k0 + KB);
    if constexpr (BF16) {
      bf8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        a[i] = *reinterpret_cast<const bf8*>(&As[buf][wm + i * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        b[j] = *reinterpret_cast<const bf8*>(&Bs[buf][wn + j * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    } else {
#pragma unroll
      for (int kk = 0; kk < KB; kk += 4) {
        float a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = As[buf][kk + (lane >> 4)][wm + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = Bs[buf][kk + (lane >> 4)][wn + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  if (d.ksplit == 1) {
    C += bz * d.sc;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
          const int col = n0 + wn + j * 16 + (lane & 15);
          if (row < d.M && col < d.N) {
            const long long off = offC<TABLE>(d, row, col);
            double v = alpha * (double)acc[i][j][r];
            if (beta != 0.0) v += beta * C[off];
            C[off] = v;
          }
        }
  } else {
    double* P = d.part + (long long)blockIdx.z * d.M * d.N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
          const int col = n0 + wn + j * 16 + (lane & 15);
          if (row < d.M && col < d.N) P[(long long)row * d.N + col] = (double)acc[i][j][r];
        }
  }
}

// C = alpha * sum_s part[s] + beta * C, partial order fixed (deterministic)
template <bool TABLE>
__global__ void splitk_reduce_kernel(double* __restrict__ C, TDesc d, double alpha, double beta,
                                     int batch) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long mn = (long long)d.M * d.N;
  if (t >= mn * batch) return;
  const long long bz = t / mn, e = t % mn;
  const int row = (int)(e / d.N), col = (int)(e % d.N);
  double s = 0.0;
  for (int p = 0; p < d.ksplit; ++p) s += d.part[(bz * d.ksplit + p) * mn + e];
  double* Cb = C + bz * d.sc;
  const long long off = offC<TABLE>(d, row, col);
  double v = alpha * s;
  if (beta != 0.0) v += beta * Cb[off];
  Cb[off] = v;
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

namespace {

// Workgroups of a kernel that the device runs at once (occupancy per CU
// times the CU count), queried once per kernel.
long long concurrent_groups(const void* fn) {
  static std::map<const void*, long long> cache;
  auto it = cache.find(fn);
  if (it != cache.end()) return it->second;
  int dev = 0, cus = 0, per = 0;
  long long slots = 512;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, 256, 0) == hipSuccess && per > 0)
    slots = (long long)per * cus;
  (void)hipGetLastError();
  cache[fn] = slots;
  return slots;
}

const void* kernel_of(int prec, int tbn, bool table) {
  if (prec == P_F64) {
    if (tbn == 32)
      return table ? (const void*)tgemm_f64_kernel<true, 32> : (const void*)tgemm_f64_kernel<false, 32>;
    if (tbn == 96)
      return table ? (const void*)tgemm_f64_kernel<true, 96> : (const void*)tgemm_f64_kernel<false, 96>;
    if (tbn == 128)
      return table ? (const void*)tgemm_f64_kernel<true, 128>
                   : (const void*)tgemm_f64_kernel<false, 128>;
    return table ? (const void*)tgemm_f64_kernel<true, 64> : (const void*)tgemm_f64_kernel<false, 64>;
  }
  if (prec == P_F32)
    return table ? (const void*)tgemm_lp_kernel<false, true> : (const void*)tgemm_lp_kernel<false, false>;
  return table ? (const void*)tgemm_lp_kernel<true, true> : (const void*)tgemm_lp_kernel<true, false>;
}

// Launch with either tables (TABLE) or strides.  A grid of fewer tiles than
// the device holds at once is split along K: the split minimises the number
// of k slices on the critical path, (full rounds of workgroups) x (slices
// per workgroup), plus a small charge per split for the partial sums.
int launch(tn_ctx* ctx, bool table, TDesc& d, int batch, const double* A, const double* B,
           double* C, double alpha, double beta, int prec) {
  // FP64: one tile across a narrow N (65..128 columns), so that the large
  // operand streams once; but with a short K (no split) the product is
  // spread over 32-column tiles when they fit in one round of workgroups
  int tbn = (prec == P_F64 && d.N > 64 && d.N <= 96) ? 96
            : (prec == P_F64 && d.N > 96 && d.N <= 128) ? 128 : BN;
  const int kstep = prec == P_BF16 ? 32 : BK;  // k slice of the kernel
  const int ktiles = (d.K + kstep - 1) / kstep;
  if (tbn > BN && ktiles < 8) {
    const long long t32 = (long long)((d.M + BM - 1) / BM) * ((d.N + 31) / 32) * batch;
    if (t32 <= concurrent_groups(kernel_of(prec, 32, table))) tbn = 32;
  }
  const long long tm = (d.M + BM - 1) / BM, tn = (d.N + tbn - 1) / tbn;
  const long long tiles = tm * tn * batch;
  int ksplit = 1;
  const long long slots = concurrent_groups(kernel_of(prec, tbn, table));
  if (tiles < slots && ktiles >= 8) {
    const int kmax = std::max(1, std::min(64, ktiles / 4));
    long long best = -1;
    for (int ks = 1; ks <= kmax; ++ks) {
      const long long rounds = (tiles * ks + slots - 1) / slots;
      const long long cost = rounds * ((ktiles + ks - 1) / ks) + ks / 4;
      if (best < 0 || cost < best) {
        best = cost;
        ksplit = ks;
      }
    }
  }
  d.ksplit = ksplit;
  d.kchunk = ((ktiles + ksplit - 1) / ksplit) * kstep;
  d.part = nullptr;
  const size_t mark = ctx->arena_off;
  if (ksplit > 1) {
    d.part = ws_alloc<double>(ctx, (size_t)ksplit * batch * d.M * d.N);
    if (!d.part) {  // no room for partials: run unsplit
      ctx->err.clear();
      ctx->arena_off = mark;
      d.ksplit = 1;
      d.kchunk = ktiles * kstep;
    }
  }
  if (d.M > 0 && d.N > 0 && (long long)batch * d.ksplit > 65535)
    TN_FAIL(ctx, TN_EINVAL, "contraction batch too large for one launch");
  dim3 grid((unsigned)tm, (unsigned)tn, (unsigned)(batch * d.ksplit));
  // Profiling: the start and stop times are stamped by the dispatches
  // themselves (the contraction kernel's start, the last kernel's end), so
  // that the measurement adds no marker packets between kernels.
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ctx->prof) {
    while (ctx->ev_pool.size() < ctx->ev_used + 2) {
      hipEvent_t e;
      // timing only: no system-scope fence (L2 write-back) at the stamps
      TN_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
      ctx->ev_pool.push_back(e);
    }
    e0 = ctx->ev_pool[ctx->ev_used];
    e1 = ctx->ev_pool[ctx->ev_used + 1];
    ctx->ev_used += 2;
    ctx->prof_flops.push_back(2.0 * (double)d.M * (double)d.N * (double)d.K * (double)batch);
    // operands read once and the result written once
    ctx->prof_bytes += 8.0 * ((double)d.M * d.K + (double)d.K * d.N + (double)d.M * d.N) * batch;
  }
  hipEvent_t stop_main = d.ksplit > 1 ? nullptr : e1;
#define TN_GO(KERNEL)                                                                          \
  hipExtLaunchKernelGGL(KERNEL, grid, dim3(256), 0, ctx->stream, e0, stop_main, 0, A, B, C, d, \
                        alpha, beta)
  if (prec == P_F64) {
    if (tbn == 32) {
      if (table) TN_GO((tgemm_f64_kernel<true, 32>)); else TN_GO((tgemm_f64_kernel<false, 32>));
    } else if (tbn == 96) {
      if (table) TN_GO((tgemm_f64_kernel<true, 96>)); else TN_GO((tgemm_f64_kernel<false, 96>));
    } else if (tbn == 128) {
      if (table) TN_GO((tgemm_f64_kernel<true, 128>)); else TN_GO((tgemm_f64_kernel<false, 128>));
    } else {
      if (table) TN_GO((tgemm_f64_kernel<true, 64>)); else TN_GO((tgemm_f64_kernel<false, 64>));
    }
  } else if (prec == P_F32) {
    if (table) TN_GO((tgemm_lp_kernel<false, true>)); else TN_GO((tgemm_lp_kernel<false, false>));
  } else {
    if (table) TN_GO((tgemm_lp_kernel<true, true>)); else TN_GO((tgemm_lp_kernel<true, false>));
  }
#undef TN_GO
  TN_HIP(ctx, hipGetLastError());
  if (d.ksplit > 1) {
    const long long tot = (long long)d.M * d.N * batch;
    const dim3 rgrid((unsigned)((tot + 255) / 256));
    if (table)
      hipExtLaunchKernelGGL(splitk_reduce_kernel<true>, rgrid, dim3(256), 0, ctx->stream, nullptr,
                            e1, 0, C, d, alpha, beta, batch);
    else
      hipExtLaunchKernelGGL(splitk_reduce_kernel<false>, rgrid, dim3(256), 0, ctx->stream,
                            nullptr, e1, 0, C, d, alpha, beta, batch);
    TN_HIP(ctx, hipGetLastError());
  }
  ctx->arena_off = mark;  // partials are consumed in stream order
  return TN_OK;
}

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
  if (prec != P_F64 && prec != P_F32 && prec != P_BF16)
    TN_FAIL(ctx, TN_EINVAL, "unknown contraction precision %d", prec);
  TDesc d;
  std::memset(&d, 0, sizeof(d));
  d.M = (int)M;
  d.N = (int)N;
  d.K = (int)K;
  // single-index groups run in strided mode, the rest through offset tables
  const bool strided = c.am.ext.size() == 1 && c.ak.ext.size() == 1 && c.bk.ext.size() == 1 &&
                       c.bn.ext.size() == 1 && c.cm.ext.size() == 1 && c.cn.ext.size() == 1;
  if (strided) {
    d.sam = c.am.str[0];
    d.sak = c.ak.str[0];
    d.sbk = c.bk.str[0];
    d.sbn = c.bn.str[0];
    d.scm = c.cm.str[0];
    d.scn = c.cn.str[0];
  } else {
    TN_TRY(table_of(ctx, c.am, &d.am));
    TN_TRY(table_of(ctx, c.ak, &d.ak));
    TN_TRY(table_of(ctx, c.bk, &d.bk));
    TN_TRY(table_of(ctx, c.bn, &d.bn));
    TN_TRY(table_of(ctx, c.cm, &d.cm));
    TN_TRY(table_of(ctx, c.cn, &d.cn));
  }
  d.sa = c.sa;
  d.sb = c.sb;
  d.sc = c.sc;
  d.a_mfast = unit_fast(c.am) || !unit_fast(c.ak);
  d.b_nfast = unit_fast(c.bn) || !unit_fast(c.bk);
  return launch(ctx, !strided, d, c.batch, A, B, C, alpha, beta, prec);
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
