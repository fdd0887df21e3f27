// Directional CTMRG on the GPU (Sec. VI B of the paper, Fig. 21(a)) and the
// reduced density matrices computed from its environment.
//
// Every move is the left move of the lattice rotated by 0, 90, 180 or 270
// degrees counter-clockwise ("frame" f).  In frame f the corner and edge
// slots k of a position are the lattice slots (k + f) mod 4 and the site
// tensor is the lattice tensor rotated f times; positions map through the
// composed rotation (x', y') = (y, -x).  All four enlarged corners of a 2x2
// block are therefore one contraction, the upper-left one, evaluated in
// frames f, f+1, f+2, f+3; the projector matrix R_u^T R_d of the row cut is
// the transpose of the ring product K = E2 E3 E0 E1 of those corners.
//
// Projectors come from the top-chi singular triplets of K, computed without
// forming K (four n x n x k products per application, n = chi D^2): block
// subspace iteration on K K^T with k = chi + oversampling columns,
// orthonormalised by shifted Cholesky-QR (three passes), Rayleigh-Ritz by a
// one-sided Jacobi SVD of the transposed k x k factor, stopped when the residual
// |K w_i - s_i v_i| of every kept triplet is below tol * s_1.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.h"
#include "nets.h"

namespace {

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------

// one counter-clockwise rotation of a site tensor: new (l,r,d,u) = old (u,d,l,r)
__global__ void rotate_site_kernel(const double* __restrict__ A, double* __restrict__ B, int d,
                                   int D) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)d * D * D * D * D;
  if (t >= tot) return;
  long long r = t;
  const int u2 = r % D; r /= D;
  const int d2 = r % D; r /= D;
  const int r2 = r % D; r /= D;
  const int l2 = r % D; r /= D;
  const int s = (int)r;
  // new[s][l2][r2][d2][u2] = old[s][l=d2][r=u2][d=r2][u=l2]
  const long long src = ((((long long)s * D + d2) * D + u2) * D + r2) * D + l2;
  B[t] = A[src];
}

__global__ void copy_cols_kernel(int n, int kin, int kout, const double* __restrict__ X,
                                 double* __restrict__ Y) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * kout) return;
  const int i = (int)(t / kout), j = (int)(t % kout);
  Y[t] = X[(long long)i * kin + j];
}

// per problem b (blockIdx.y) and kept column i < chi: |Y[:,i] - S[i] V[:,i]|
// (Y, V: [batch][n][k], S: [batch][k], colres: [batch][chi])
__global__ __launch_bounds__(256) void resid_kernel(int n, int k, int chi,
                                                    const double* __restrict__ Y,
                                                    const double* __restrict__ V,
                                                    const double* __restrict__ S,
                                                    double* __restrict__ colres) {
  const int j = blockIdx.x;
  const long long b = blockIdx.y;
  Y += b * n * k;
  V += b * n * k;
  __shared__ double part[4];
  double a = 0.0;
  const double s = S[b * k + j];
  for (int i = threadIdx.x; i < n; i += 256) {
    const double r = Y[(long long)i * k + j] - s * V[(long long)i * k + j];
    a += r * r;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) colres[b * chi + j] = sqrt(part[0] + part[1] + part[2] + part[3]);
}

// out = max over problems of (max_i colres[b][i]) / S[b][0]
__global__ void max_over_kernel(const double* __restrict__ colres, int chi, int batch,
                                const double* __restrict__ S, int k, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double r = 0.0;
  for (int b = 0; b < batch; ++b) {
    double m = 0.0;
    for (int i = 0; i < chi; ++i) m = fmax(m, colres[b * chi + i]);
    const double s0 = S[(long long)b * k];
    r = fmax(r, s0 > 0.0 ? m / s0 : m);
  }
  *out = r;
}

// At[b] = A[b]^T for a batch of k x k row-major matrices
__global__ __launch_bounds__(256) void transpose_sq_kernel(int k, long long total,
                                                           const double* __restrict__ A,
                                                           double* __restrict__ At) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= total) return;
  const long long kk = (long long)k * k, b = t / kk;
  const int r = (int)(t - b * kk), i = r / k, j = r - i * k;
  At[b * kk + (long long)j * k + i] = A[t];
}

// sign convention on the kept left singular vectors of M (= W): the first
// entry within a relative 1e-8 of the largest magnitude is made positive; the
// matching columns of V flip with them
__global__ __launch_bounds__(256) void signfix_kernel(int n, int ldw, double* __restrict__ W,
                                                      int ldv, double* __restrict__ V) {
  const int j = blockIdx.x;
  __shared__ double red[4];
  __shared__ int redi[4];
  double best = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) best = fmax(best, fabs(W[(long long)i * ldw + j]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) best = fmax(best, __shfl_xor(best, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
  __syncthreads();
  const double mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  const double thr = (1.0 - 1e-8) * mx;
  int idx = 0x7fffffff;
  for (int i = threadIdx.x; i < n; i += 256)
    if (fabs(W[(long long)i * ldw + j]) >= thr) {
      idx = i;
      break;
    }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) idx = min(idx, __shfl_xor(idx, o, 64));
  if ((threadIdx.x & 63) == 0) redi[threadIdx.x >> 6] = idx;
  __syncthreads();
  const int first = min(min(redi[0], redi[1]), min(redi[2], redi[3]));
  const double sg = (first < n && W[(long long)first * ldw + j] < 0.0) ? -1.0 : 1.0;
  if (sg < 0.0)
    for (int i = threadIdx.x; i < n; i += 256) {
      W[(long long)i * ldw + j] = -W[(long long)i * ldw + j];
      V[(long long)i * ldv + j] = -V[(long long)i * ldv + j];
    }
}

// spectra: normalise each row of S to unit l2 norm, compare with prev,
// out = max over rows of the l2 difference; prev <- normalised S
__global__ void spectra_delta_kernel(const double* __restrict__ S, double* __restrict__ prev,
                                     int rows, int chi, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double dmax = 0.0;
  for (int r = 0; r < rows; ++r) {
    double nrm = 0.0;
    for (int i = 0; i < chi; ++i) nrm += S[r * chi + i] * S[r * chi + i];
    nrm = sqrt(nrm);
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    double dd = 0.0;
    for (int i = 0; i < chi; ++i) {
      const double v = S[r * chi + i] * inv;
      const double e = v - prev[r * chi + i];
      dd += e * e;
      prev[r * chi + i] = v;
    }
    dmax = fmax(dmax, sqrt(dd));
  }
  *out = dmax;
}

__global__ void trace_normalize_kernel(double* __restrict__ R, int dim, long long stride) {
  double* r = R + (long long)blockIdx.x * stride;
  __shared__ double tr;
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < dim; ++i) t += r[i * dim + i];
    tr = t;
  }
  __syncthreads();
  const double inv = 1.0 / tr;
  for (int i = threadIdx.x; i < dim * dim; i += blockDim.x) r[i] *= inv;
}

__global__ void finite_check_kernel(const double* __restrict__ x, long long n, int* flag) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(x[i])) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------

struct Frames {
  int Lx[4], Ly[4];
  std::vector<int> pos[4];  // pos[f][y*Lx_f + x] = lattice position
  int at(int f, int x, int y) const {
    const int lx = Lx[f], ly = Ly[f];
    x = ((x % lx) + lx) % lx;
    y = ((y % ly) + ly) % ly;
    return pos[f][y * lx + x];
  }
};

Frames make_frames(int Lx, int Ly) {
  Frames F;
  F.Lx[0] = Lx;
  F.Ly[0] = Ly;
  F.pos[0].resize(Lx * Ly);
  for (int p = 0; p < Lx * Ly; ++p) F.pos[0][p] = p;
  for (int f = 1; f < 4; ++f) {
    const int ox = F.Lx[f - 1], oy = F.Ly[f - 1];
    F.Lx[f] = oy;
    F.Ly[f] = ox;
    F.pos[f].resize(Lx * Ly);
    for (int yn = 0; yn < ox; ++yn)
      for (int xn = 0; xn < oy; ++xn) {
        const int x = ((-yn) % ox + ox) % ox, y = xn;
        F.pos[f][yn * oy + xn] = F.pos[f - 1][y * ox + x];
      }
  }
  return F;
}

struct Geo {
  int Lx, Ly, D, d, nsite, chi, npos, n;
  int prec = P_F64;       // bulk contractions: corners, K products, projectors, renormalisation
  double svd_tol = 1e-13; // residual tolerance of the projector SVD (relative to s_1)
  int svd_maxit = 40;
  std::vector<int> cell;
  Frames F;
  const double* arot[4];  // rotated site tensors [nsite][d][D^4]
  double* C;
  double* T;
  long long csz() const { return (long long)chi * chi; }
  long long tsz() const { return (long long)chi * D * D * chi; }
  double* Cp(int p, int k) const { return C + ((long long)p * 4 + (k & 3)) * csz(); }
  double* Tp(int p, int k) const { return T + ((long long)p * 4 + (k & 3)) * tsz(); }
  const double* site(int f, int p) const {
    return arot[f & 3] + (long long)cell[p] * d * D * D * D * D;
  }
};

// ---------------------------------------------------------------------------
// Absorption of one site into a half-contracted network, ket and bra layers in
// one kernel:
//   Out[c,a,rk,dk,rb,db] = sum_{s,lk,uk,lb,ub} In[c,a,lk,uk,lb,ub]
//                              A[s,lk,rk,dk,uk] A[s,lb,rb,db,ub]
// (the site-tensor step of the enlarged corners and of the edge
// renormalisation, Sec. VI B).  Read as matrices over index pairs of
// P = D^2 entries, with Am[s] the P x P matrix Am[s][(l,u)][(r,dn)] =
// A[s,l,r,dn,u], the product is two chained small GEMMs per (c, a) pair:
//   T[(l,u')][s][R1] = sum_K1 In[K1][(l,u')] Am[s][K1][R1]    (ket layer)
//   Out[R1][R2]      = sum_{s,L} T[L][s][R1] Am[s][L][R2]      (bra layer)
// A workgroup takes G = 4 consecutive (c, a) pairs and one wave per 16 rows
// of the stacked G*P rows.  Both products are FP64 MFMA 16x16x4 tiles with
// the same B operand, Am[s] staged in LDS; the ket result passes to the bra product through LDS (transposed), one
// physical index s at a time, so the 2 d D^4-entry intermediate of every
// pair never reaches HBM.  In and Out are addressed by strides, so the same
// kernel serves both index layouts.
// ---------------------------------------------------------------------------
typedef double dv4 __attribute__((ext_vector_type(4)));

struct AbsorbDesc {
  long long in_c, in_a, in_lk, in_uk, in_lb, in_ub;
  long long out_c, out_a, out_rk, out_dk, out_rb, out_db;
  int nc, na, d;
};

constexpr int ABS_G = 4;

template <int D>
constexpr int absorb_threads() {
  return 64 * ((ABS_G * D * D + 15) / 16);
}

// D = 6: three 9-wave workgroups per CU need 7 waves per SIMD (at most 72
// VGPRs) and at most 53 KB of LDS each
template <int D>
constexpr int absorb_min_waves() {
  return D == 6 ? 7 : 1;
}

// Output layouts the store knows: ABS_STRIDED stores each lane's own entries
// (any strides); ABS_RUN_B and ABS_RUN_D stage the workgroup's tile in LDS
// and store it in runs of G D^2 consecutive doubles, when the four pairs are
// consecutive in the output with stride D^2 and (rb, rk) (corner layout) or
// (db, dk) (edge layout) are the two fastest output indices.
enum { ABS_STRIDED = 0, ABS_RUN_B = 1, ABS_RUN_D = 2 };

template <int D, int LAYOUT>
__global__ __launch_bounds__(absorb_threads<D>(), absorb_min_waves<D>()) void absorb_kernel(
    const double* __restrict__ In, const double* __restrict__ A, double* __restrict__ Out,
    AbsorbDesc g) {
  constexpr int P = D * D;
  constexpr int ROWS = ABS_G * P;
  constexpr int NJ = (P + 15) / 16;  // 16-column blocks over P
  constexpr int NQ = (P + 3) / 4;    // k-steps of 4 over P
  constexpr int S = P % 2 == 0 ? P + 1 : P + 2;  // LDS row stride (odd)
  __shared__ double Ts[ROWS * S];
  __shared__ double Bs[NQ * 4 * S];
  const int lane = threadIdx.x & 63, blk = threadIdx.x >> 6;
  const int hi = lane >> 4, lo = lane & 15;
  const long long npair = (long long)g.nc * g.na;
  // consecutive workgroups go to different XCDs (each with its own L2), and
  // neighbouring pair blocks share the cache lines of In: give the blocks
  // that one XCD runs (physical ids b, b + 8, b + 16, ...) consecutive pairs
  long long bid = blockIdx.x;
  {
    const long long per = gridDim.x / 8;
    if (bid < per * 8) bid = (bid % 8) * per + bid / 8;
  }
  const long long p0 = bid * ABS_G;
  // operand-A row of this lane: m = 16 blk + lo, i.e. pair m / P, index pair m % P
  const int mA = 16 * blk + lo;
  const int aA = mA / P, LA = mA % P;
  const bool rowA = mA < ROWS;
  const bool okA = rowA && p0 + aA < npair;
  double inA[NQ];
  {
    long long base = 0;
    if (okA) {
      const long long pr = p0 + aA, c = pr / g.na, a = pr % g.na;
      base = c * g.in_c + a * g.in_a + (long long)(LA / D) * g.in_lb + (long long)(LA % D) * g.in_ub;
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int k1 = 4 * q + hi;
      inA[q] = (okA && k1 < P)
                   ? In[base + (long long)(k1 / D) * g.in_lk + (long long)(k1 % D) * g.in_uk]
                   : 0.0;
    }
  }
  dv4 acc2[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) acc2[j] = dv4{0.0, 0.0, 0.0, 0.0};
  for (int s = 0; s < g.d; ++s) {
    // Am[s] into LDS, zero-padded to NQ*4 rows: the B operand of both
    // products, Bs[4q + lane/16][16j + lane%16]; the columns past P are
    // not stored, their operand lanes read zero
    for (int t = threadIdx.x; t < NQ * 4 * P; t += blockDim.x) {
      const int row = t / P, col = t % P;
      Bs[row * S + col] = row < P ? A[(long long)s * P * P + (row / D) * D * P + (col / D) * P +
                                      (col % D) * D + (row % D)]
                                  : 0.0;
    }
    __syncthreads();
    // ket layer: rows (pair, l, u') of this wave, one 16-column block of R1
    // at a time (one accumulator live beside acc2 and inA keeps the kernel
    // within the registers of two workgroups per CU)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      dv4 acc1 = dv4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const double b = 16 * j + lo < P ? Bs[(4 * q + hi) * S + 16 * j + lo] : 0.0;
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(inA[q], b, acc1, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * blk + hi + 4 * r;
        if (row < ROWS && 16 * j + lo < P) Ts[row * S + 16 * j + lo] = acc1[r];
      }
    }
    __syncthreads();
    // bra layer: rows (pair, R1) of this wave, k over (l, u') of the same pair
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int L = 4 * q + hi;
      const double a2 = (rowA && L < P) ? Ts[(aA * P + L) * S + LA] : 0.0;
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const double b = 16 * j + lo < P ? Bs[(4 * q + hi) * S + 16 * j + lo] : 0.0;
        acc2[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, b, acc2[j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  if (LAYOUT == ABS_STRIDED) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * blk + hi + 4 * r;
      const int ap = row / P, R1 = row % P;
      const long long pr = p0 + ap;
      if (row >= ROWS || pr >= npair) continue;
      const long long c = pr / g.na, a = pr % g.na;
      const long long base = c * g.out_c + a * g.out_a + (long long)(R1 / D) * g.out_rk +
                             (long long)(R1 % D) * g.out_dk;
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int R2 = 16 * j + lo;
        if (R2 < P)
          Out[base + (long long)(R2 / D) * g.out_rb + (long long)(R2 % D) * g.out_db] =
              acc2[j][r];
      }
    }
    return;
  }
  // stage the tile Os[(pair, R1)][R2] in Ts (free after the last barrier of
  // the loop), then store it in runs: element e = ((y1 D + y0) G + p) D^2 +
  // x1 D + x0 with (x0, x1) = (rb, rk) or (db, dk) and (y0, y1) the other two
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 16 * blk + hi + 4 * r;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int R2 = 16 * j + lo;
      if (row < ROWS && R2 < P) Ts[row * S + R2] = acc2[j][r];
    }
  }
  __syncthreads();
  // the G pairs are consecutive in the output (checked on the host), so the
  // tile's base is that of its first pair
  const long long c0 = p0 / g.na, a0 = p0 % g.na;
  const long long base0 = c0 * g.out_c + a0 * g.out_a;
  const long long ystride0 = LAYOUT == ABS_RUN_B ? g.out_db : g.out_rb;
  const long long ystride1 = LAYOUT == ABS_RUN_B ? g.out_dk : g.out_rk;
  const int nvalid = (int)min((long long)ABS_G, npair - p0);
  for (int e = threadIdx.x; e < ROWS * P; e += blockDim.x) {
    const int x = e % P, q = e / P;  // x = x1 D + x0, contiguous in the output
    const int p = q % ABS_G, y = q / ABS_G;
    if (p >= nvalid) continue;
    const int x0 = x % D, x1 = x / D, y0 = y % D, y1 = y / D;
    // R1 = (rk, dk), R2 = (rb, db)
    const int R1 = LAYOUT == ABS_RUN_B ? x1 * D + y1 : y1 * D + x1;
    const int R2 = LAYOUT == ABS_RUN_B ? x0 * D + y0 : y0 * D + x0;
    Out[base0 + (long long)p * P + x + y0 * ystride0 + y1 * ystride1] =
        Ts[(p * P + R1) * S + R2];
  }
}

// Fused absorption for D = 2..6 in FP64; returns false (nothing launched)
// for other bond dimensions or precisions, where the caller runs the two
// products as separate contractions.
template <int D>
void absorb_launch(tn_ctx* ctx, int layout, dim3 grid, const double* In, const double* A,
                   double* Out, const AbsorbDesc& g) {
  if (layout == ABS_RUN_B)
    hipLaunchKernelGGL((absorb_kernel<D, ABS_RUN_B>), grid, dim3(absorb_threads<D>()), 0,
                       ctx->stream, In, A, Out, g);
  else if (layout == ABS_RUN_D)
    hipLaunchKernelGGL((absorb_kernel<D, ABS_RUN_D>), grid, dim3(absorb_threads<D>()), 0,
                       ctx->stream, In, A, Out, g);
  else
    hipLaunchKernelGGL((absorb_kernel<D, ABS_STRIDED>), grid, dim3(absorb_threads<D>()), 0,
                       ctx->stream, In, A, Out, g);
}

bool absorb_site(tn_ctx* ctx, int D, int prec, const double* In, const double* A, double* Out,
                 const AbsorbDesc& g) {
  if (prec != P_F64 || D < 2 || D > 6) return false;
  const long long npair = (long long)g.nc * g.na;
  if (npair <= 0) return true;
  const dim3 grid((unsigned)((npair + ABS_G - 1) / ABS_G));
  // runs need the G pairs of a workgroup consecutive in the output: na a
  // multiple of G (the pairs share c), a-stride D^2, and the two fastest
  // output indices of one of the two kinds
  const long long P = (long long)D * D;
  int layout = ABS_STRIDED;
  if (g.na % ABS_G == 0 && g.out_a == P) {
    if (g.out_rb == 1 && g.out_rk == D && g.out_db % (ABS_G * P) == 0 &&
        g.out_dk % (ABS_G * P) == 0)
      layout = ABS_RUN_B;
    else if (g.out_db == 1 && g.out_dk == D && g.out_rb % (ABS_G * P) == 0 &&
             g.out_rk % (ABS_G * P) == 0)
      layout = ABS_RUN_D;
  }
  switch (D) {
    case 2: absorb_launch<2>(ctx, layout, grid, In, A, Out, g); break;
    case 3: absorb_launch<3>(ctx, layout, grid, In, A, Out, g); break;
    case 4: absorb_launch<4>(ctx, layout, grid, In, A, Out, g); break;
    case 5: absorb_launch<5>(ctx, layout, grid, In, A, Out, g); break;
    default: absorb_launch<6>(ctx, layout, grid, In, A, Out, g); break;
  }
  return true;
}

// ---------------------------------------------------------------------------
// contractions
// ---------------------------------------------------------------------------

// Upper-left enlarged corner
// E[(a, dk, db), (b, rk, rb)] = sum C[g,h] T1[h,uk,ub,b] T4[a,lk,lb,g] A[s,lk,rk,dk,uk] A[s,lb,rb,db,ub]
// scratch: X1 chi*D2*chi, X2 chi*D2*D2*chi, X3 chi*chi*d*D2*D2.
int corner_ul(tn_ctx* ctx, const Geo& g, const double* Cc, const double* T1, const double* T4,
              const double* A, double* E, double* X1, double* X2, double* X3) {
  const long long chi = g.chi, D = g.D, d = g.d, D2 = D * D, D4 = D2 * D2, n = g.n;
  TN_TRY(gemm(ctx, (int)(chi * D2), (int)chi, (int)chi, T4, (int)chi, false, Cc, (int)chi, false,
              X1, (int)chi, 1.0, 0.0, 1, 0, 0, 0, g.prec));
  TN_TRY(gemm(ctx, (int)(chi * D2), (int)(D2 * chi), (int)chi, X1, (int)chi, false, T1,
              (int)(D2 * chi), false, X2, (int)(D2 * chi), 1.0, 0.0, 1, 0, 0, 0, g.prec));
  {
    // X2[a, lk, lb, uk, ub, b] -> E[(a, dk, db), (b, rk, rb)], both layers at once
    AbsorbDesc ad;
    ad.in_c = D4 * chi, ad.in_a = 1, ad.in_lk = D2 * D * chi, ad.in_uk = D * chi;
    ad.in_lb = D2 * chi, ad.in_ub = chi;
    ad.out_c = D2 * n, ad.out_a = D2, ad.out_rk = D, ad.out_dk = D * n, ad.out_rb = 1;
    ad.out_db = n;
    ad.nc = (int)chi, ad.na = (int)chi, ad.d = (int)d;
    if (absorb_site(ctx, (int)D, g.prec, X2, A, E, ad)) {
      TN_HIP(ctx, hipGetLastError());
      return TN_OK;
    }
  }
  TN_TRY(tc_run(ctx, nets::corner_ket(chi, D, d), X2, A, X3, 1.0, 0.0, g.prec));
  TN_TRY(tc_run(ctx, nets::corner_bra(chi, D, d, n), X3, A, E, 1.0, 0.0, g.prec));
  return TN_OK;
}

// corner j of the block in frame f: frame-(f+j) upper-left corner at lattice position p
int corner_of(tn_ctx* ctx, const Geo& g, int fj, int p, double* E, double* X1, double* X2,
              double* X3) {
  return corner_ul(ctx, g, g.Cp(p, fj), g.Tp(p, fj), g.Tp(p, fj + 3), g.site(fj, p), E, X1, X2, X3);
}

// `batch` independent projector problems (the row cuts of one move): the
// corners of problem b are E[j] + b n^2; t1, t2 are [batch][n][k] scratch.
struct TopK {
  int n, k, chi, batch;
  int prec;  // precision of the products with the corners
  const double* E[4];
  double *t1, *t2;
};

// Y = K X with K = E2 E3 E0 E1, per problem
int applyK(tn_ctx* ctx, const TopK& t, const double* X, double* Y) {
  const int n = t.n, k = t.k, B = t.batch;
  const long long sE = (long long)n * n, sX = (long long)n * k;
  TN_TRY(gemm(ctx, n, k, n, t.E[1], n, false, X, k, false, t.t1, k, 1.0, 0.0, B, sE, sX, sX, t.prec));
  TN_TRY(gemm(ctx, n, k, n, t.E[0], n, false, t.t1, k, false, t.t2, k, 1.0, 0.0, B, sE, sX, sX, t.prec));
  TN_TRY(gemm(ctx, n, k, n, t.E[3], n, false, t.t2, k, false, t.t1, k, 1.0, 0.0, B, sE, sX, sX, t.prec));
  TN_TRY(gemm(ctx, n, k, n, t.E[2], n, false, t.t1, k, false, Y, k, 1.0, 0.0, B, sE, sX, sX, t.prec));
  return TN_OK;
}

// Y = K^T X, per problem
int applyKT(tn_ctx* ctx, const TopK& t, const double* X, double* Y) {
  const int n = t.n, k = t.k, B = t.batch;
  const long long sE = (long long)n * n, sX = (long long)n * k;
  TN_TRY(gemm(ctx, n, k, n, t.E[2], n, true, X, k, false, t.t1, k, 1.0, 0.0, B, sE, sX, sX, t.prec));
  TN_TRY(gemm(ctx, n, k, n, t.E[3], n, true, t.t1, k, false, t.t2, k, 1.0, 0.0, B, sE, sX, sX, t.prec));
  TN_TRY(gemm(ctx, n, k, n, t.E[0], n, true, t.t2, k, false, t.t1, k, 1.0, 0.0, B, sE, sX, sX, t.prec));
  TN_TRY(gemm(ctx, n, k, n, t.E[1], n, true, t.t1, k, false, Y, k, 1.0, 0.0, B, sE, sX, sX, t.prec));
  return TN_OK;
}

// Column scaling by 1 / max(s_j, floor * s_0) per problem (floor keeps
// columns below the FP64 resolution of the block at unit scale instead of
// blowing them up); X = Src scaled (Src may be X), [batch][n][k]; s and sc
// [batch][k].
__global__ void inv_scale_cols_kernel(int n, int k, int batch, const double* Src, double* X,
                                      const double* s, double floor_rel, double* sc) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < (long long)batch * k) {
    const long long b = t / k;
    sc[t] = fmax(s[t], floor_rel * s[b * k]);
  }
  if (t >= (long long)batch * n * k) return;
  const long long b = t / ((long long)n * k);
  const int j = (int)(t % k);
  const double* sb = s + b * k;
  X[t] = Src[t] / fmax(sb[j], floor_rel * sb[0]);
}

// R <- R diag(sc) per problem (R [batch][k][k], sc [batch][k])
__global__ void right_scale_kernel(int k, int batch, double* R, const double* sc) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)batch * k * k) return;
  const long long b = t / ((long long)k * k);
  R[t] *= sc[b * k + t % k];
}

// Orthonormalise the columns of X ([batch] blocks of n x k) in place:
// Cholesky-QR passes, the first `nshift` of them shifted (shifted
// Cholesky-QR, Fukaya et al., SIAM J. Sci. Comput. 2020), `npass` in total.
// R ([batch][k][k], optional) with X_in = Q R.  info[pass * batch + b]
// receives the Cholesky status of each pass and problem.
int cholqr_passes(tn_ctx* ctx, int n, int k, int batch, double* X, double* Rout, double* tmp,
                  int* info, int npass, int nshift) {
  // scratch is reused by the next call: later kernels on the same stream
  // run after these, so releasing the arena slice here is safe
  const size_t mark = ctx->arena_off;
  const long long kk = (long long)k * k, nk = (long long)n * k;
  double* G = ws_alloc<double>(ctx, (size_t)batch * kk);
  double* R = ws_alloc<double>(ctx, (size_t)batch * kk * npass);
  double* Ri = ws_alloc<double>(ctx, (size_t)batch * kk);
  double* Racc = ws_alloc<double>(ctx, (size_t)batch * kk);
  if (!Racc) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted in cholqr");
  const double u = 1.1102230246251565e-16;
  double* src = X;
  double* dst = tmp;
  for (int pass = 0; pass < npass; ++pass) {
    TN_TRY(gemm(ctx, k, k, n, src, k, true, src, k, false, G, k, 1.0, 0.0, batch, nk, nk, kk));
    const double shift = pass < nshift ? 11.0 * ((double)n * k + (double)k * (k + 1)) * u : 0.0;
    TN_TRY(cholesky_inv(ctx, k, G, shift, R + (size_t)pass * batch * kk, Ri, info + pass * batch,
                        batch));
    TN_TRY(gemm(ctx, n, k, k, src, k, false, Ri, k, false, dst, k, 1.0, 0.0, batch, nk, kk, nk));
    std::swap(src, dst);
  }
  if (src != X)
    TN_HIP(ctx, hipMemcpyAsync(X, src, (size_t)batch * nk * sizeof(double),
                               hipMemcpyDeviceToDevice, ctx->stream));
  if (Rout) {
    // R = R_last ... R_1, the partial products alternating between Racc and
    // Rout so that the last lands in Rout
    const double* acc = R + (size_t)(npass - 1) * batch * kk;
    if (npass == 1)
      TN_HIP(ctx, hipMemcpyAsync(Rout, acc, (size_t)batch * kk * 8, hipMemcpyDeviceToDevice,
                                 ctx->stream));
    for (int pass = npass - 2; pass >= 0; --pass) {
      double* dst = pass % 2 == 0 ? Rout : Racc;
      TN_TRY(gemm(ctx, k, k, k, acc, k, false, R + (size_t)pass * batch * kk, k, false, dst, k,
                  1.0, 0.0, batch, kk, kk, kk));
      acc = dst;
    }
  }
  ctx->arena_off = mark;
  return TN_OK;
}

// X = Src + c_b Z per problem b, with c_b = 1e-10 |Src_b|_F / sqrt(n k): the
// random directions Z complete a block of lower rank than its column count
// (one workgroup per problem)
__global__ __launch_bounds__(256) void fill_deficient_kernel(int n, int k,
                                                             const double* __restrict__ Src,
                                                             const double* __restrict__ Z,
                                                             double* __restrict__ X) {
  __shared__ double red[4];
  const long long nk = (long long)n * k, off = (long long)blockIdx.x * nk;
  double a = 0.0;
  for (long long i = threadIdx.x; i < nk; i += 256) a += Src[off + i] * Src[off + i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  const double c = 1e-10 * sqrt((red[0] + red[1] + red[2] + red[3]) / (double)nk);
  for (long long i = threadIdx.x; i < nk; i += 256) X[off + i] = Src[off + i] + c * Z[off + i];
}

// Robust orthonormalisation of [batch] blocks: optional column pre-scaling by
// `scale` (the current Ritz values, which makes a Ritz-ordered block nearly
// orthonormal), then Cholesky-QR; if any pass of any problem breaks down,
// the original blocks are redone with two shifted passes followed by two
// plain ones.
int orth_robust(tn_ctx* ctx, int n, int k, int batch, double* X, const double* scale,
                double* Rout, double* tmp, double* save, int* info) {
  const size_t mark = ctx->arena_off;
  double* sc = ws_alloc<double>(ctx, (size_t)batch * k);
  if (!sc) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted in orth_robust");
  const long long tot = (long long)batch * n * k;
  if (scale) {
    hipLaunchKernelGGL(inv_scale_cols_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                       ctx->stream, n, k, batch, X, X, scale, 1e-15, sc);
    TN_HIP(ctx, hipGetLastError());
  }
  TN_HIP(ctx, hipMemcpyAsync(save, X, (size_t)tot * 8, hipMemcpyDeviceToDevice, ctx->stream));
  const int ninfo = 4 * batch;
  TN_HIP(ctx, hipMemsetAsync(info, 0, ninfo * sizeof(int), ctx->stream));
  // a pre-scaled block is close to orthonormal: two plain passes give
  // orthogonality to rounding; otherwise shifted Cholesky-QR3
  if (scale)
    TN_TRY(cholqr_passes(ctx, n, k, batch, X, Rout, tmp, info, 2, 0));
  else
    TN_TRY(cholqr_passes(ctx, n, k, batch, X, Rout, tmp, info, 3, 1));
  std::vector<int> h(ninfo);
  TN_HIP(ctx, hipMemcpyAsync(h.data(), info, ninfo * sizeof(int), hipMemcpyDeviceToHost,
                             ctx->stream));
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  bool bad = false;
  for (int v : h) bad = bad || v != 0;
  if (bad) {
    TN_HIP(ctx, hipMemcpyAsync(X, save, (size_t)tot * 8, hipMemcpyDeviceToDevice, ctx->stream));
    TN_HIP(ctx, hipMemsetAsync(info, 0, ninfo * sizeof(int), ctx->stream));
    TN_TRY(cholqr_passes(ctx, n, k, batch, X, Rout, tmp, info, 4, 2));
    TN_HIP(ctx, hipMemcpyAsync(h.data(), info, ninfo * sizeof(int), hipMemcpyDeviceToHost,
                               ctx->stream));
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
    bad = false;
    for (int v : h) bad = bad || v != 0;
  }
  if (bad) {
    // the block has fewer independent directions than columns (a projector
    // problem of low numerical rank, e.g. a nearly product state): complete
    // it with random directions at 1e-10 of its scale, orthonormalise, and
    // take R = Q^T X of the block itself, so that X = Q R still holds
    double* Z = ws_alloc<double>(ctx, (size_t)tot);
    if (!Z) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted in orth_robust");
    TN_TRY(fill_random(ctx, Z, tot, 0x5EEDF111ULL + (unsigned long long)tot));
    hipLaunchKernelGGL(fill_deficient_kernel, dim3(batch), dim3(256), 0, ctx->stream, n, k, save,
                       Z, X);
    TN_HIP(ctx, hipGetLastError());
    TN_HIP(ctx, hipMemsetAsync(info, 0, ninfo * sizeof(int), ctx->stream));
    TN_TRY(cholqr_passes(ctx, n, k, batch, X, nullptr, tmp, info, 4, 2));
    TN_HIP(ctx, hipMemcpyAsync(h.data(), info, ninfo * sizeof(int), hipMemcpyDeviceToHost,
                               ctx->stream));
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int v : h)
      if (v) TN_FAIL(ctx, TN_ENUMERIC, "Cholesky-QR breakdown in the projector SVD");
    if (Rout) {
      const long long nk = (long long)n * k, kk = (long long)k * k;
      TN_TRY(gemm(ctx, k, k, n, X, k, true, save, k, false, Rout, k, 1.0, 0.0, batch, nk, nk,
                  kk));
    }
  }
  if (scale && Rout) {
    const long long tk = (long long)batch * k * k;
    hipLaunchKernelGGL(right_scale_kernel, dim3((unsigned)((tk + 255) / 256)), dim3(256), 0,
                       ctx->stream, k, batch, Rout, sc);
    TN_HIP(ctx, hipGetLastError());
  }
  ctx->arena_off = mark;
  return TN_OK;
}

// Orthonormalisation of a Ritz-ordered block without a host round trip: the
// column pre-scaling by `scale` makes the block nearly orthonormal, and two
// plain Cholesky-QR passes follow.  The Cholesky status of every pass and
// problem goes to info[4 * batch] and is checked by the caller later; a
// breakdown is then redone through orth_robust.  The block is read from src
// when given (X is then written, not read).
int orth_fast(tn_ctx* ctx, int n, int k, int batch, double* X, const double* scale,
              double* Rout, double* tmp, int* info, const double* src = nullptr) {
  const size_t mark = ctx->arena_off;
  double* sc = ws_alloc<double>(ctx, (size_t)batch * k);
  if (!sc) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted in orth_fast");
  const long long tot = (long long)batch * n * k;
  hipLaunchKernelGGL(inv_scale_cols_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                     ctx->stream, n, k, batch, src ? src : X, X, scale, 1e-15, sc);
  TN_HIP(ctx, hipGetLastError());
  TN_TRY(cholqr_passes(ctx, n, k, batch, X, Rout, tmp, info, 2, 0));
  if (Rout) {
    const long long tk = (long long)batch * k * k;
    hipLaunchKernelGGL(right_scale_kernel, dim3((unsigned)((tk + 255) / 256)), dim3(256), 0,
                       ctx->stream, k, batch, Rout, sc);
    TN_HIP(ctx, hipGetLastError());
  }
  ctx->arena_off = mark;
  return TN_OK;
}

struct SvdStats {
  long long iters = 0, calls = 0, unconverged = 0, explicit_calls = 0;
};

// Top-chi singular triplets of K_b = V_b S_b W_b^T for every problem b:
// Vout, Wout [batch][n][chi], Sout [batch][chi].  warmQ [batch][n][k] and
// warmS [batch][k]: optional start bases and their Ritz values (in/out).
int topk_svd(tn_ctx* ctx, TopK& t, double* warmQ, double* warmS, bool warm_valid, double* Vout,
             double* Sout, double* Wout, double tol, int maxit, unsigned long long seed,
             SvdStats* st) {
  const int n = t.n, k = t.k, chi = t.chi, B = t.batch;
  const size_t nk = (size_t)n * k;
  const long long nchi = (long long)n * chi;
  if (n <= 256) {
    // small problems: form K and take its full one-sided Jacobi SVD
    double* Km = ws_alloc<double>(ctx, (size_t)n * n);
    double* K2 = ws_alloc<double>(ctx, (size_t)n * n);
    double* Uf = ws_alloc<double>(ctx, (size_t)n * n);
    double* Vf = ws_alloc<double>(ctx, (size_t)n * n);
    double* Sf = ws_alloc<double>(ctx, (size_t)n);
    if (!Sf) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted in topk_svd");
    const long long sE = (long long)n * n;
    for (int b = 0; b < B; ++b) {
      TN_TRY(gemm(ctx, n, n, n, t.E[0] + b * sE, n, false, t.E[1] + b * sE, n, false, Km, n, 1.0,
                  0.0, 1, 0, 0, 0, t.prec));
      TN_TRY(gemm(ctx, n, n, n, t.E[3] + b * sE, n, false, Km, n, false, K2, n, 1.0, 0.0, 1, 0, 0,
                  0, t.prec));
      TN_TRY(gemm(ctx, n, n, n, t.E[2] + b * sE, n, false, K2, n, false, Km, n, 1.0, 0.0, 1, 0, 0,
                  0, t.prec));
      TN_TRY(jacobi_svd(ctx, 1, n, n, Km, n, 0, Uf, n, 0, Sf, 0, Vf, n, 0));
      hipLaunchKernelGGL(copy_cols_kernel, dim3((unsigned)((nchi + 255) / 256)), dim3(256), 0,
                         ctx->stream, n, n, chi, Uf, Vout + b * nchi);
      hipLaunchKernelGGL(copy_cols_kernel, dim3((unsigned)((nchi + 255) / 256)), dim3(256), 0,
                         ctx->stream, n, n, chi, Vf, Wout + b * nchi);
      TN_HIP(ctx, hipMemcpyAsync(Sout + b * chi, Sf, chi * sizeof(double),
                                 hipMemcpyDeviceToDevice, ctx->stream));
      hipLaunchKernelGGL(signfix_kernel, dim3(chi), dim3(256), 0, ctx->stream, n, chi,
                         Wout + b * nchi, chi, Vout + b * nchi);
      TN_HIP(ctx, hipGetLastError());
    }
    if (st) st->explicit_calls += B;
    return TN_OK;
  }
  const size_t bnk = (size_t)B * nk, bkk = (size_t)B * k * k;
  double* Q = ws_alloc<double>(ctx, bnk);
  double* Bm = ws_alloc<double>(ctx, bnk);
  double* Y = ws_alloc<double>(ctx, bnk);
  double* Wb = ws_alloc<double>(ctx, bnk);
  double* Vr = ws_alloc<double>(ctx, bnk);
  double* tmp = ws_alloc<double>(ctx, bnk);
  double* save = ws_alloc<double>(ctx, bnk);
  double* R = ws_alloc<double>(ctx, bkk);
  double* Rt = ws_alloc<double>(ctx, bkk);
  double* UR = ws_alloc<double>(ctx, bkk);
  double* VR = ws_alloc<double>(ctx, bkk);
  double* S = ws_alloc<double>(ctx, (size_t)B * k);
  double* Sprev = ws_alloc<double>(ctx, (size_t)B * k);
  double* colres = ws_alloc<double>(ctx, (size_t)B * chi);
  double* res = ws_alloc<double>(ctx, 1);
  int* info = ws_alloc<int>(ctx, 8 * B);
  int* info_b = ws_alloc<int>(ctx, 4 * B);  // orth of K^T Q, this iteration
  int* info_q = ws_alloc<int>(ctx, 4 * B);  // orth of the previous K W
  constexpr int MAX_PLAIN = 3;
  int* info_p = ws_alloc<int>(ctx, 2 * MAX_PLAIN * 2 * B);  // orths of the plain steps
  double* Ysave = ws_alloc<double>(ctx, bnk);
  double* Zk = ws_alloc<double>(ctx, bnk);
  if (!Zk) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted in topk_svd");
  const long long kk = (long long)k * k, snk = (long long)nk;
  bool have_s = false;
  if (warmQ && warm_valid) {
    TN_HIP(ctx, hipMemcpyAsync(Q, warmQ, bnk * sizeof(double), hipMemcpyDeviceToDevice,
                               ctx->stream));
    TN_HIP(ctx, hipMemcpyAsync(Sprev, warmS, (size_t)B * k * sizeof(double),
                               hipMemcpyDeviceToDevice, ctx->stream));
    have_s = true;
  } else {
    TN_TRY(fill_random(ctx, Q, (long long)bnk, seed));
  }
  TN_TRY(orth_robust(ctx, n, k, B, Q, nullptr, nullptr, tmp, save, info));
  // One host round trip per iteration: the orthonormalisations of a warm,
  // Ritz-scaled block run without checking their Cholesky status at once;
  // the status comes back with the residual, and a breakdown redoes the
  // iteration through the robust path (from the saved K W of the previous
  // iteration when the current basis is the one that broke down).
  // Between Rayleigh-Ritz steps the iteration may take plain steps,
  // Q <- orth(K orth(K^T Q)) scaled by the last Ritz values, with no SVD of
  // the k x k factor and no host round trip: after the third iteration the
  // residual's rate of decrease predicts how many steps remain, and all but
  // the last of them (at most MAX_PLAIN) are plain.  Their Cholesky status is
  // checked with the next Rayleigh-Ritz step; a breakdown restarts from the
  // last checked block on the robust path, without further plain steps.
  bool q_pending = false, robust = false, allow_plain = true, s_current = true;
  int retries = 0, plain_left = 0, plain_done = 0, it_prev = 0;
  int it = 0;
  double hres = 1.0, r_prev = -1.0;
  // Cholesky status read back per Rayleigh-Ritz step: 2B (basis) + 2B
  // (pending orth) + MAX_PLAIN 4B (plain steps) ints after 8 doubles
  if (8 * sizeof(double) + (size_t)(4 + 4 * MAX_PLAIN) * B * sizeof(int) >
      TN_HOST_SCRATCH * sizeof(double))
    TN_FAIL(ctx, TN_EINVAL, "%d row cuts exceed the projector SVD's status buffer", B);
  int* hinfo = reinterpret_cast<int*>(ctx->host_scratch + 8);
  for (it = 1; it <= maxit; ++it) {
    if (plain_left > 0 && allow_plain && have_s && !robust) {
      int* ip = info_p + plain_done * 4 * B;
      TN_TRY(applyKT(ctx, t, Q, Bm));
      TN_TRY(orth_fast(ctx, n, k, B, Bm, Sprev, nullptr, tmp, ip));
      TN_TRY(applyK(ctx, t, Bm, Q));
      TN_TRY(orth_fast(ctx, n, k, B, Q, Sprev, nullptr, tmp, ip + 2 * B));
      --plain_left;
      ++plain_done;
      continue;
    }
    TN_TRY(applyKT(ctx, t, Q, Bm));
    const bool fast = have_s && !robust;
    if (fast)
      TN_TRY(orth_fast(ctx, n, k, B, Bm, Sprev, R, tmp, info_b));
    else
      TN_TRY(orth_robust(ctx, n, k, B, Bm, have_s ? Sprev : nullptr, R, tmp, save, info));
    // R = UR S VR^T by the one-sided Jacobi SVD of R^T = VR S UR^T (its
    // normalised columns are VR, its accumulated rotations UR).  From a warm
    // start R is diag(S) plus entries eps s_j above the diagonal: in the
    // columns of R every pair starts at cosine eps, in its rows pair (i, j)
    // at eps s_j / s_i, so only pairs of close Ritz values need rotating
    // (fewer sweeps, the QR preconditioning of one-sided Jacobi).
    const long long bkk_l = (long long)bkk;
    hipLaunchKernelGGL(transpose_sq_kernel, dim3((unsigned)((bkk_l + 255) / 256)), dim3(256), 0,
                       ctx->stream, k, bkk_l, R, Rt);
    TN_HIP(ctx, hipGetLastError());
    // The Ritz rotation UR only turns the basis inside span(Bm), so K Bm can
    // be formed while the SVD of R (a few workgroups) runs on the side
    // stream; then K Wb = (K Bm) UR.
    if (!jacobi_svd_needs_workspace(k, k)) {
      TN_TRY(side_stream_ready(ctx));
      TN_HIP(ctx, hipEventRecord(ctx->ev_fork, ctx->stream));
      TN_HIP(ctx, hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0));
      hipStream_t main_stream = ctx->stream;
      ctx->stream = ctx->side;
      const int rc = jacobi_svd(ctx, B, k, k, Rt, k, kk, VR, k, kk, S, k, UR, k, kk);
      ctx->stream = main_stream;
      if (rc != TN_OK) return rc;
      TN_HIP(ctx, hipEventRecord(ctx->ev_join, ctx->side));
      TN_TRY(applyK(ctx, t, Bm, Zk));
      TN_HIP(ctx, hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0));
      TN_TRY(gemm(ctx, n, k, k, Bm, k, false, UR, k, false, Wb, k, 1.0, 0.0, B, snk, kk, snk));
      TN_TRY(gemm(ctx, n, k, k, Q, k, false, VR, k, false, Vr, k, 1.0, 0.0, B, snk, kk, snk));
      TN_TRY(gemm(ctx, n, k, k, Zk, k, false, UR, k, false, Y, k, 1.0, 0.0, B, snk, kk, snk));
    } else {
      TN_TRY(jacobi_svd(ctx, B, k, k, Rt, k, kk, VR, k, kk, S, k, UR, k, kk));
      TN_TRY(gemm(ctx, n, k, k, Bm, k, false, UR, k, false, Wb, k, 1.0, 0.0, B, snk, kk, snk));
      TN_TRY(gemm(ctx, n, k, k, Q, k, false, VR, k, false, Vr, k, 1.0, 0.0, B, snk, kk, snk));
      TN_TRY(applyK(ctx, t, Wb, Y));
    }
    s_current = true;
    hipLaunchKernelGGL(resid_kernel, dim3(chi, B), dim3(256), 0, ctx->stream, n, k, chi, Y, Vr, S,
                       colres);
    hipLaunchKernelGGL(max_over_kernel, dim3(1), dim3(1), 0, ctx->stream, colres, chi, B, S, k,
                       res);
    TN_HIP(ctx, hipMemcpyAsync(ctx->host_scratch, res, sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
    if (fast)
      TN_HIP(ctx, hipMemcpyAsync(hinfo, info_b, 2 * B * sizeof(int), hipMemcpyDeviceToHost,
                                 ctx->stream));
    if (q_pending)
      TN_HIP(ctx, hipMemcpyAsync(hinfo + 2 * B, info_q, 2 * B * sizeof(int),
                                 hipMemcpyDeviceToHost, ctx->stream));
    if (plain_done)
      TN_HIP(ctx, hipMemcpyAsync(hinfo + 4 * B, info_p, plain_done * 4 * B * sizeof(int),
                                 hipMemcpyDeviceToHost, ctx->stream));
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
    bool bad_b = false, bad_q = false;
    for (int i = 0; i < 2 * B; ++i) {
      bad_b = bad_b || (fast && hinfo[i] != 0);
      bad_q = bad_q || (q_pending && hinfo[2 * B + i] != 0);
    }
    for (int i = 0; i < plain_done * 4 * B; ++i) bad_q = bad_q || hinfo[4 * B + i] != 0;
    if (plain_done && bad_q) allow_plain = false;
    plain_done = 0;
    if (bad_q || bad_b) {
      if (++retries > 2) TN_FAIL(ctx, TN_ENUMERIC, "Cholesky-QR breakdown in the projector SVD");
      if (bad_q) {  // the basis of this iteration was not orthonormal
        TN_HIP(ctx, hipMemcpyAsync(Q, Ysave, bnk * sizeof(double), hipMemcpyDeviceToDevice,
                                   ctx->stream));
        TN_TRY(orth_robust(ctx, n, k, B, Q, Sprev, nullptr, tmp, save, info));
      }
      q_pending = false;
      robust = true;
      --it;
      continue;
    }
    // after a breakdown the block stays on the robust path for the rest of
    // this problem: a nearly rank-deficient K (a product-like state) breaks
    // every fast orthonormalisation, and falling back to it would spend the
    // retries
    q_pending = false;
    const double hprev = hres;
    hres = ctx->host_scratch[0];
    if (!std::isfinite(hres)) TN_FAIL(ctx, TN_ENUMERIC, "non-finite residual in the projector SVD");
    if (hres <= tol || it == maxit) break;
    // the rounding floor lies above tol: the residual has stopped falling
    if (it >= 3 && hres <= 30.0 * tol && hres > 0.7 * hprev) break;
    // plain steps until the predicted last one (the drop of the first
    // iteration, from the warm start, says nothing about the rate)
    if (it >= 3 && r_prev > 0.0 && hres < r_prev) {
      const double rho = std::min(0.7, std::max(0.02, std::pow(hres / r_prev, 1.0 / (it - it_prev))));
      const int m = (int)std::ceil(std::log(tol / hres) / std::log(rho));
      plain_left = std::min(std::max(m - 1, 0), std::min(MAX_PLAIN, maxit - it - 1));
    }
    r_prev = hres;
    it_prev = it;
    // K Wb is kept (as Ysave) for a redo, and the Ritz values become the
    // scaling of the next iteration, by exchanging buffers: the next Y and S
    // are written in full before they are read
    std::swap(Y, Ysave);
    std::swap(S, Sprev);
    s_current = false;
    if (robust) {
      TN_HIP(ctx, hipMemcpyAsync(Q, Ysave, bnk * sizeof(double), hipMemcpyDeviceToDevice,
                                 ctx->stream));
      TN_TRY(orth_robust(ctx, n, k, B, Q, Sprev, nullptr, tmp, save, info));
      q_pending = false;
    } else {
      TN_TRY(orth_fast(ctx, n, k, B, Q, Sprev, nullptr, tmp, info_q, Ysave));
      q_pending = true;
    }
    have_s = true;
  }
  if (!s_current) std::swap(S, Sprev);  // the last Ritz values
  if (st) {
    st->iters += (long long)it * B;
    st->calls += B;
    if (hres > tol) st->unconverged += B;
  }
  if (warmQ) {
    TN_HIP(ctx, hipMemcpyAsync(warmQ, Vr, bnk * sizeof(double), hipMemcpyDeviceToDevice,
                               ctx->stream));
    TN_HIP(ctx, hipMemcpyAsync(warmS, S, (size_t)B * k * sizeof(double), hipMemcpyDeviceToDevice,
                               ctx->stream));
  }
  // the kept columns of every problem: rows of all problems at once
  const long long tot = (long long)B * nchi;
  hipLaunchKernelGGL(copy_cols_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                     ctx->stream, B * n, k, chi, Vr, Vout);
  hipLaunchKernelGGL(copy_cols_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                     ctx->stream, B * n, k, chi, Wb, Wout);
  for (int b = 0; b < B; ++b) {
    TN_HIP(ctx, hipMemcpyAsync(Sout + b * chi, S + (size_t)b * k, chi * sizeof(double),
                               hipMemcpyDeviceToDevice, ctx->stream));
    hipLaunchKernelGGL(signfix_kernel, dim3(chi), dim3(256), 0, ctx->stream, n, chi,
                       Wout + b * nchi, chi, Vout + b * nchi);
  }
  TN_HIP(ctx, hipGetLastError());
  return TN_OK;
}

struct MoveBufs {
  double* E[4];           // [Ly][n][n] each: corner j of every row cut
  double *X1, *X2, *X3;
  double *P, *PtT;        // [Ly][n][chi]
  double *V, *W, *S;      // [Ly][n][chi], [Ly][n][chi], [Ly][chi]
  double *G1;             // [Ly][n][chi]
  double *t1, *t2;        // [Ly][n][k]
  double *Cn1, *Tn4, *Cn4;  // new tensors [Ly][...]
  double* CT;             // chi*D2*chi
  double* warm;           // per frame, column and row: start basis [n][k] and Ritz values [k]
  int k;
};

// left move in frame f at frame column x
int left_move(tn_ctx* ctx, const Geo& g, int f, int x, MoveBufs& b, SvdStats* st, bool* warm_ok) {
  const Frames& F = g.F;
  const int Lyf = F.Ly[f], Lxf = F.Lx[f];
  const int n = g.n, chi = g.chi, D = g.D, d = g.d;
  const long long D2 = (long long)D * D;
  const long long nchi = (long long)n * chi, nn = (long long)n * n;
  // the four enlarged corners of every row cut of column x
  for (int y = 0; y < Lyf; ++y) {
    const int ptl = F.at(f, x, y), ptr = F.at(f, x + 1, y);
    const int pbr = F.at(f, x + 1, y + 1), pbl = F.at(f, x, y + 1);
    TN_TRY(corner_of(ctx, g, f + 0, ptl, b.E[0] + y * nn, b.X1, b.X2, b.X3));
    TN_TRY(corner_of(ctx, g, f + 1, ptr, b.E[1] + y * nn, b.X1, b.X2, b.X3));
    TN_TRY(corner_of(ctx, g, f + 2, pbr, b.E[2] + y * nn, b.X1, b.X2, b.X3));
    TN_TRY(corner_of(ctx, g, f + 3, pbl, b.E[3] + y * nn, b.X1, b.X2, b.X3));
  }
  // one batched top-chi SVD for all row cuts
  TopK t;
  t.n = n;
  t.k = b.k;
  t.chi = chi;
  t.batch = Lyf;
  t.prec = g.prec;
  for (int j = 0; j < 4; ++j) t.E[j] = b.E[j];
  t.t1 = b.t1;
  t.t2 = b.t2;
  // warm slots: frame-major, then column, then row (rows of a column adjacent)
  const size_t slot0 = (size_t)f * (Lxf * Lyf) + (size_t)x * Lyf;
  double* wQ = b.warm ? b.warm + slot0 * ((size_t)n * b.k + b.k) : nullptr;
  double* wS = wQ ? wQ + (size_t)Lyf * n * b.k : nullptr;
  bool wv = wQ != nullptr;
  for (int y = 0; y < Lyf && wv; ++y) wv = warm_ok[slot0 + y];
  const size_t mark = ctx->arena_off;
  TN_TRY(topk_svd(ctx, t, wQ, wS, wv, b.V, b.S, b.W, g.svd_tol, g.svd_maxit,
                  0x5DEECE66DULL * (slot0 + 1), st));
  ctx->arena_off = mark;
  if (wQ)
    for (int y = 0; y < Lyf; ++y) warm_ok[slot0 + y] = true;
  // P = E3^T (E2^T V) S^-1/2 ; Pt^T = E0 (E1 W) S^-1/2, all rows at once
  TN_TRY(gemm(ctx, n, chi, n, b.E[2], n, true, b.V, chi, false, b.G1, chi, 1.0, 0.0, Lyf, nn,
              nchi, nchi, g.prec));
  TN_TRY(gemm(ctx, n, chi, n, b.E[3], n, true, b.G1, chi, false, b.P, chi, 1.0, 0.0, Lyf, nn,
              nchi, nchi, g.prec));
  TN_TRY(gemm(ctx, n, chi, n, b.E[1], n, false, b.W, chi, false, b.G1, chi, 1.0, 0.0, Lyf, nn,
              nchi, nchi, g.prec));
  TN_TRY(gemm(ctx, n, chi, n, b.E[0], n, false, b.G1, chi, false, b.PtT, chi, 1.0, 0.0, Lyf, nn,
              nchi, nchi, g.prec));
  for (int y = 0; y < Lyf; ++y) {
    TN_TRY(scale_columns(ctx, n, chi, b.P + y * nchi, chi, b.S + y * chi, 1));
    TN_TRY(scale_columns(ctx, n, chi, b.PtT + y * nchi, chi, b.S + y * chi, 1));
  }
  const long long csz = (long long)chi * chi, tsz = (long long)chi * D2 * chi;
  for (int y = 0; y < Lyf; ++y) {
    const int src = F.at(f, x, y), s1 = F.at(f, x, y + 1);
    const double* P = b.P + (size_t)y * nchi;
    const double* PtTy = b.PtT + (size_t)y * nchi;
    const double* PtTm = b.PtT + (size_t)((y - 1 + Lyf) % Lyf) * nchi;
    // C1 of (x+1, y+1) = P_y^T (C1 T1)(x, y+1)
    TN_TRY(gemm(ctx, chi, (int)(D2 * chi), chi, g.Cp(s1, f), chi, false, g.Tp(s1, f),
                (int)(D2 * chi), false, b.CT, (int)(D2 * chi), 1.0, 0.0, 1, 0, 0, 0, g.prec));
    TN_TRY(gemm(ctx, chi, chi, n, P, chi, true, b.CT, chi, false, b.Cn1 + y * csz, chi, 1.0, 0.0, 1, 0, 0,
                0, g.prec));
    // C4 of (x+1, y) = [T3 C4](x, y) Pt_y^T, Z[a3, (b4, k, b)]
    {
      TN_TRY(tc_run(ctx, nets::t3_c4(chi, D, n), g.Tp(src, f + 2), g.Cp(src, f + 3), b.CT, 1.0,
                    0.0, g.prec));
      TN_TRY(gemm(ctx, chi, chi, n, b.CT, n, false, PtTy, chi, false, b.Cn4 + y * csz, chi, 1.0,
                  0.0, 1, 0, 0, 0, g.prec));
    }
    // T4 of (x+1, y) = Pt_{y-1} (T4 a a)(x, y) P_y
    {
      const double* T4 = g.Tp(src, f + 3);
      const double* A = g.site(f, src);
      const long long nn = n;
      double* Y1 = b.X2;  // chi * D2 * n
      double* Y2 = b.X3;  // chi * d * D4 * chi
      double* Y3 = b.X2;  // chi * D2 * n (Y1 is dead by then)
      // Y1[c, uk, ub, a, lk, lb] = sum_b PtT[(b,uk,ub), c] T4[a, lk, lb, b]
      TN_TRY(tc_run(ctx, nets::edge_pt(chi, D, nn), PtTm, T4, Y1, 1.0, 0.0, g.prec));
      AbsorbDesc ad;  // Y1 -> Y3 with both layers in one kernel
      ad.in_c = D2 * nn, ad.in_a = D2, ad.in_lk = D, ad.in_uk = D * nn, ad.in_lb = 1;
      ad.in_ub = nn;
      ad.out_c = D2 * nn, ad.out_a = D2, ad.out_rk = D * nn, ad.out_dk = D, ad.out_rb = nn;
      ad.out_db = 1;
      ad.nc = chi, ad.na = chi, ad.d = d;
      // out of place: Y3 may not overwrite Y1 while other workgroups read it
      const bool fused = absorb_site(ctx, D, g.prec, Y1, A, b.X3, ad);
      if (fused) {
        TN_HIP(ctx, hipGetLastError());
        Y3 = b.X3;
      }
      // unfused: Y2 = Y1 A (ket layer), Y3 = Y2 A (bra layer)
      if (!fused) {
        TN_TRY(tc_run(ctx, nets::edge_ket(chi, D, d, nn), Y1, A, Y2, 1.0, 0.0, g.prec));
        TN_TRY(tc_run(ctx, nets::edge_bra(chi, D, d, nn), Y2, A, Y3, 1.0, 0.0, g.prec));
      }
      // T4new[e, rk, rb, c] = sum_i Y3[c, rk, rb, i] P[i, e]
      TN_TRY(tc_run(ctx, nets::edge_p(chi, D, nn), Y3, P, b.Tn4 + y * tsz, 1.0, 0.0, g.prec));
    }
  }
  // write back and normalise
  for (int y = 0; y < Lyf; ++y) {
    const int dst = F.at(f, x + 1, y), d1 = F.at(f, x + 1, y + 1);
    TN_TRY(frob_normalize_to(ctx, b.Cn1 + y * csz, g.Cp(d1, f), csz, nullptr));
    TN_TRY(frob_normalize_to(ctx, b.Tn4 + y * tsz, g.Tp(dst, f + 3), tsz, nullptr));
    TN_TRY(frob_normalize_to(ctx, b.Cn4 + y * csz, g.Cp(dst, f + 3), csz, nullptr));
  }
  return TN_OK;
}

int check_geometry(tn_ctx* ctx, int Lx, int Ly, int D, int d, int nsite, const double* sites,
                   const int* cell, int chi, const void* C, const void* T) {
  if (!ctx) return TN_EINVAL;
  if (Lx < 1 || Ly < 1 || D < 1 || d < 1 || nsite < 1 || chi < 1)
    TN_FAIL(ctx, TN_EINVAL, "sizes must be positive (Lx=%d Ly=%d D=%d d=%d nsite=%d chi=%d)",
            Lx, Ly, D, d, nsite, chi);
  if (Lx * Ly > 64) TN_FAIL(ctx, TN_EINVAL, "cell larger than 64 positions");
  if (!sites || !cell || !C || !T) TN_FAIL(ctx, TN_EINVAL, "null pointer argument");
  for (int p = 0; p < Lx * Ly; ++p)
    if (cell[p] < 0 || cell[p] >= nsite)
      TN_FAIL(ctx, TN_EINVAL, "cell[%d] = %d out of range [0, %d)", p, cell[p], nsite);
  const long long n = (long long)chi * D * D;
  if (n > 32768) TN_FAIL(ctx, TN_EINVAL, "chi*D*D = %lld too large", n);
  return TN_OK;
}

int setup_geo(tn_ctx* ctx, Geo& g, int Lx, int Ly, int D, int d, int nsite, const double* sites,
              const int* cell, int chi, double* C, double* T) {
  g.Lx = Lx;
  g.Ly = Ly;
  g.D = D;
  g.d = d;
  g.nsite = nsite;
  g.chi = chi;
  g.npos = Lx * Ly;
  g.n = chi * D * D;
  g.cell.assign(cell, cell + Lx * Ly);
  g.F = make_frames(Lx, Ly);
  g.C = C;
  g.T = T;
  const long long asz = (long long)nsite * d * D * D * D * D;
  g.arot[0] = sites;
  const double* prev = sites;
  for (int f = 1; f < 4; ++f) {
    double* r = ws_alloc<double>(ctx, asz);
    if (!r) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted (rotated sites)");
    for (int s = 0; s < nsite; ++s) {
      const long long one = (long long)d * D * D * D * D;
      hipLaunchKernelGGL(rotate_site_kernel, dim3((unsigned)((one + 255) / 256)), dim3(256), 0,
                         ctx->stream, prev + s * one, r + s * one, d, D);
    }
    TN_HIP(ctx, hipGetLastError());
    g.arot[f] = r;
    prev = r;
  }
  return TN_OK;
}

size_t move_bytes(const Geo& g, int k, bool warm) {
  const size_t chi = g.chi, D = g.D, d = g.d, D2 = D * D, n = g.n;
  const size_t Lm = std::max(g.Lx, g.Ly);
  size_t b = 0;
  auto add = [&](size_t cnt) { b += ((cnt * 8 + 255) / 256) * 256; };
  for (int j = 0; j < 4; ++j) add(Lm * n * n);
  add(chi * D2 * chi);
  add(std::max(chi * D2 * D2 * chi, chi * D2 * n));
  add(chi * chi * d * D2 * D2);
  add(Lm * n * chi);  // P
  add(Lm * n * chi);  // PtT
  add(Lm * n * chi);  // V
  add(Lm * n * chi);  // W
  add(Lm * chi);      // S
  add(Lm * n * chi);  // G1
  add(Lm * n * k);    // t1
  add(Lm * n * k);    // t2
  add(Lm * chi * chi);
  add(Lm * chi * D2 * chi);
  add(Lm * chi * chi);
  add(chi * D2 * chi);
  (void)warm;
  add(Lm * (16 * n * k + 64 * (size_t)k * k));  // split-K partials of the n x n x k products
  // topk_svd scratch (explicit path for n <= 256, subspace path otherwise)
  add(std::max(Lm * 9 * n * k, 4 * n * n + n));
  add(Lm * 4 * k * k);  // R, R^T, UR, VR
  add(Lm * (4 * k + chi) + 64);
  add(Lm * 16 + 64);
  add(64);                                        // status of the plain steps
  add(256);                                       // partial sums of the normalisations
  add(Lm * (8 * k * k + k) + 64);                 // Cholesky-QR passes (one alive at a time)
  add(Lm * (2 * std::max((size_t)k * k, n * n) + 2 * (size_t)k * k));  // jacobi work
  // rotated sites
  add(3 * (size_t)g.nsite * d * D2 * D2);
  // spectra
  add(8 * (size_t)g.npos * chi * chi);
  return b + (1 << 20);
}

int alloc_move_bufs(tn_ctx* ctx, const Geo& g, MoveBufs& b, bool warm) {
  const size_t chi = g.chi, D = g.D, d = g.d, D2 = D * D, n = g.n;
  const size_t Lm = std::max(g.Lx, g.Ly);
  for (int j = 0; j < 4; ++j) b.E[j] = ws_alloc<double>(ctx, Lm * n * n);
  b.X1 = ws_alloc<double>(ctx, chi * D2 * chi);
  b.X2 = ws_alloc<double>(ctx, std::max(chi * D2 * D2 * chi, chi * D2 * n));
  b.X3 = ws_alloc<double>(ctx, chi * chi * d * D2 * D2);
  b.P = ws_alloc<double>(ctx, Lm * n * chi);
  b.PtT = ws_alloc<double>(ctx, Lm * n * chi);
  b.V = ws_alloc<double>(ctx, Lm * n * chi);
  b.W = ws_alloc<double>(ctx, Lm * n * chi);
  b.S = ws_alloc<double>(ctx, Lm * chi);
  b.G1 = ws_alloc<double>(ctx, Lm * n * chi);
  b.t1 = ws_alloc<double>(ctx, Lm * n * b.k);
  b.t2 = ws_alloc<double>(ctx, Lm * n * b.k);
  b.Cn1 = ws_alloc<double>(ctx, Lm * chi * chi);
  b.Tn4 = ws_alloc<double>(ctx, Lm * chi * D2 * chi);
  b.Cn4 = ws_alloc<double>(ctx, Lm * chi * chi);
  b.CT = ws_alloc<double>(ctx, chi * D2 * chi);
  b.warm = warm ? ws_alloc<double>(ctx, (size_t)4 * g.npos * (n * b.k + b.k)) : nullptr;
  if (!b.CT || (warm && !b.warm)) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted (move buffers)");
  return TN_OK;
}

int pick_k(int n, int chi) {
  int k = chi + std::max(16, chi / 4);
  k = (k + 15) / 16 * 16;
  return std::min(k, n);
}

int finite_or_fail(tn_ctx* ctx, const double* x, long long n, const char* what) {
  int* flag = ws_alloc<int>(ctx, 1);
  if (!flag) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted");
  TN_HIP(ctx, hipMemsetAsync(flag, 0, sizeof(int), ctx->stream));
  hipLaunchKernelGGL(finite_check_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     ctx->stream, x, n, flag);
  int h = 0;
  TN_HIP(ctx, hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (h) TN_FAIL(ctx, TN_ENUMERIC, "non-finite values in %s", what);
  return TN_OK;
}

// ---------------------------------------------------------------------------
// reduced density matrices
// ---------------------------------------------------------------------------

// Left half of the horizontal two-site network in frame f at lattice
// position p: L[t, s, s', rk, rb, b] (t = T1.b, b = T3.a in frame f).
int half_left(tn_ctx* ctx, const Geo& g, int f, int p, double* L, double* X1, double* X2,
              double* X3, double* X4, double* Y) {
  const long long chi = g.chi, D = g.D, d = g.d, D2 = D * D, n = g.n;
  const double* C1 = g.Cp(p, f);
  const double* T1 = g.Tp(p, f);
  const double* T4 = g.Tp(p, f + 3);
  const double* C4 = g.Cp(p, f + 3);
  const double* T3 = g.Tp(p, f + 2);
  const double* A = g.site(f, p);
  TN_TRY(gemm(ctx, (int)(chi * D2), (int)chi, (int)chi, T4, (int)chi, false, C1, (int)chi, false,
              X1, (int)chi, 1.0, 0.0));
  TN_TRY(gemm(ctx, (int)(chi * D2), (int)(D2 * chi), (int)chi, X1, (int)chi, false, T1,
              (int)(D2 * chi), false, X2, (int)(D2 * chi), 1.0, 0.0));
  // X3[e][t][rk][dk][s][lb][ub] as in the corner, then the bra layer with s' open
  TN_TRY(tc_run(ctx, nets::corner_ket(chi, D, d), X2, A, X3, 1.0, 0.0));
  TN_TRY(tc_run(ctx, nets::half_bra(chi, D, d, n), X3, A, X4, 1.0, 0.0));
  // Y[(b, dk, db), e] = T3[(b,dk,db), f] C4[f, e]
  TN_TRY(gemm(ctx, (int)(chi * D2), (int)chi, (int)chi, T3, (int)chi, false, C4, (int)chi, false,
              Y, (int)chi, 1.0, 0.0));
  // L[(t,s,s',rk,rb), b] = sum_{e,dk,db} X4[..., e, dk, db] Y[b, dk, db, e]
  TN_TRY(tc_run(ctx, nets::half_close(chi, D, d, n), X4, Y, L, 1.0, 0.0));
  return TN_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// public entry points (C ABI wrappers live in abi.hip)
// ---------------------------------------------------------------------------

// Bulk precision of a phase: the contraction precision, and the projector
// SVD tolerance and iteration cap that its rounding allows (the residual of
// a reduced-precision product cannot drop below its rounding level).
void set_precision(Geo& g, int prec) {
  g.prec = prec;
  if (prec == P_F64) {
    // the residual's rounding floor grows with the length n of the vectors
    // (measured 7e-14 to 9e-14 s_1 at n = 2592, about 0.3 n u): the target
    // is 1e-13 or 0.4 n u, whichever is larger (2.7e-13 at n = 8192, where
    // 1e-13 lay below the floor and every problem ended on the stagnation
    // rule)
    g.svd_tol = std::max(1e-13, 0.4 * (double)g.n * 1.1102230246251565e-16);
    g.svd_maxit = 40;
  } else if (prec == P_F32) {
    g.svd_tol = 2e-5;
    g.svd_maxit = 12;
  } else {
    g.svd_tol = 2e-2;
    g.svd_maxit = 6;
  }
}

int ctmrg_run_impl(tn_ctx* ctx, int Lx, int Ly, int D, int d, int nsite, const double* sites,
                   const int* cell, int chi, double* C, double* T, int max_iter, double tol,
                   int n_moves, int first_dir, int* iters, double* delta, int prec,
                   int n_polish) {
  TN_TRY(check_geometry(ctx, Lx, Ly, D, d, nsite, sites, cell, chi, C, T));
  Geo g;
  const int n = chi * D * D;
  const int k = pick_k(n, chi);
  {
    Geo tmp;
    tmp.Lx = Lx;
    tmp.Ly = Ly;
    tmp.D = D;
    tmp.d = d;
    tmp.nsite = nsite;
    tmp.chi = chi;
    tmp.npos = Lx * Ly;
    tmp.n = n;
    TN_TRY(ws_reserve(ctx, move_bytes(tmp, k, true)));
  }
  ws_reset(ctx);
  TN_TRY(setup_geo(ctx, g, Lx, Ly, D, d, nsite, sites, cell, chi, C, T));
  MoveBufs b;
  b.k = k;
  TN_TRY(alloc_move_bufs(ctx, g, b, false));
  // projector start bases persist in the context across calls with the same
  // geometry (a converging CTMRG changes them little between iterations)
  char key[160];
  snprintf(key, sizeof(key), "ctm-warm:%d:%d:%d:%d:%d:%d", Lx, Ly, D, d, chi, k);
  for (int p = 0; p < Lx * Ly; ++p) snprintf(key + strlen(key), sizeof(key) - strlen(key), ":%d", cell[p]);
  void* wptr = nullptr;
  bool fresh = false;
  TN_TRY(keep_buffer(ctx, key, (size_t)4 * g.npos * ((size_t)n * k + k) * sizeof(double), &wptr,
                     &fresh));
  b.warm = static_cast<double*>(wptr);
  std::vector<char>& flags = ctx->keep_flags[key];
  if (fresh || flags.size() != (size_t)4 * g.npos) flags.assign((size_t)4 * g.npos, 0);
  bool* wok = reinterpret_cast<bool*>(flags.data());
  SvdStats st;
  set_precision(g, prec);
  const size_t base = ctx->arena_off;
  if (n_moves > 0) {
    // exact move count, in iteration order starting at first_dir
    int done = 0, f = first_dir & 3;
    while (done < n_moves) {
      for (int x = 0; x < g.F.Lx[f] && done < n_moves; ++x, ++done) {
        ctx->arena_off = base;
        TN_TRY(left_move(ctx, g, f, x, b, &st, wok));
      }
      f = (f + 1) & 3;
    }
    TN_TRY(finite_or_fail(ctx, C, (long long)g.npos * 4 * g.csz(), "corners"));
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->moves += n_moves;
    ctx->svd_calls += st.calls;
    ctx->svd_iters += st.iters;
    ctx->svd_unconverged += st.unconverged;
    ctx->svd_explicit += st.explicit_calls;
    return TN_OK;
  }
  // iterate to convergence
  const int rows = g.npos * 4;
  double* Sprev = ws_alloc<double>(ctx, (size_t)rows * chi);
  double* Sc = ws_alloc<double>(ctx, (size_t)rows * chi);
  double* dd = ws_alloc<double>(ctx, 1);
  if (!dd) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted (spectra)");
  const size_t base2 = ctx->arena_off;
  // spectra of the starting corners
  TN_TRY(jacobi_svd(ctx, rows, chi, chi, C, chi, g.csz(), nullptr, 0, 0, Sc, chi, nullptr, 0, 0));
  hipLaunchKernelGGL(spectra_delta_kernel, dim3(1), dim3(1), 0, ctx->stream, Sc, Sprev, rows, chi,
                     dd);
  // Reduced bulk precision: iterate until delta reaches the precision's
  // switch level sw (1e-6 FP32, 1e-3 BF16), or stops improving at the
  // precision's noise floor (after five iterations, the best delta of the
  // last three is not below 0.7 times the best before them); then FP64
  // iterations, at least n_polish of them and until delta < tol.  At most
  // max_iter iterations in all (plus n_polish if the reduced phase used them
  // up).  FP64 throughout: until delta < tol or max_iter.  Either way the
  // FP64 iterations also stop when they stall (below).
  const double sw = prec == P_F32 ? 1e-6 : (prec == P_BF16 ? 1e-3 : tol);
  const int polish = prec == P_F64 ? 0 : std::max(0, n_polish);
  int it = 0, done_it = 0, fp64_it = 0;
  double hd = INFINITY;
  std::vector<double> hist, hist64;
  const int cap = max_iter + polish;
  for (it = 1; it <= cap; ++it) {
    if (g.prec != P_F64) {
      bool stalled = false;
      const int nh = (int)hist.size();
      if (nh >= 5) {
        double recent = INFINITY, before = INFINITY;
        for (int i = 0; i < nh; ++i) (i >= nh - 3 ? recent : before) =
            std::min(i >= nh - 3 ? recent : before, hist[i]);
        stalled = recent > 0.7 * before;
      }
      if (hd < sw || stalled || it > max_iter) set_precision(g, P_F64);
    }
    for (int f = 0; f < 4; ++f)
      for (int x = 0; x < g.F.Lx[f]; ++x) {
        ctx->arena_off = base2;
        TN_TRY(left_move(ctx, g, f, x, b, &st, wok));
      }
    ctx->arena_off = base2;
    TN_TRY(jacobi_svd(ctx, rows, chi, chi, C, chi, g.csz(), nullptr, 0, 0, Sc, chi, nullptr, 0, 0));
    hipLaunchKernelGGL(spectra_delta_kernel, dim3(1), dim3(1), 0, ctx->stream, Sc, Sprev, rows,
                       chi, dd);
    TN_HIP(ctx, hipMemcpyAsync(ctx->host_scratch, dd, sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
    hd = ctx->host_scratch[0];
    hist.push_back(hd);
    ++done_it;
    if (g.prec == P_F64) {
      ++fp64_it;
      hist64.push_back(hd);
    }
    if (!std::isfinite(hd)) TN_FAIL(ctx, TN_ENUMERIC, "non-finite corner spectra");
    if (g.prec == P_F64 && hd < tol && fp64_it >= polish) break;
    if (prec == P_F64 && it >= max_iter) break;
    // FP64 stall: after 20 FP64 iterations, the best delta of the last 10
    // is not below 0.9 times the best before them (progress that slow, a
    // rate above 0.9895 per iteration, would not reach tol within hundreds
    // of iterations; a cut through a dense part of the projector spectrum
    // keeps delta fluctuating without a trend)
    const int nf = (int)hist64.size();
    if (g.prec == P_F64 && fp64_it >= polish && nf >= 20) {
      double recent = INFINITY, before = INFINITY;
      for (int i = 0; i < nf; ++i) {
        if (i >= nf - 10) recent = std::min(recent, hist64[i]);
        else before = std::min(before, hist64[i]);
      }
      if (recent > 0.9 * before) break;
    }
  }
  if (iters) *iters = done_it;
  if (delta) *delta = hd;
  ctx->moves += (long long)done_it * (2 * (g.F.Lx[0] + g.F.Lx[1]));
  ctx->svd_calls += st.calls;
  ctx->svd_iters += st.iters;
  ctx->svd_unconverged += st.unconverged;
  ctx->svd_explicit += st.explicit_calls;
  return (hd < tol) ? TN_OK : TN_NOT_CONVERGED;
}

int ipeps_rdms_impl(tn_ctx* ctx, int Lx, int Ly, int D, int d, int nsite, const double* sites,
                    const int* cell, int chi, const double* C, const double* T, double* rho1,
                    double* rhoh, double* rhov) {
  TN_TRY(check_geometry(ctx, Lx, Ly, D, d, nsite, sites, cell, chi, C, T));
  if (!rho1 || !rhoh || !rhov) TN_FAIL(ctx, TN_EINVAL, "null output pointer");
  const size_t chi_ = chi, D_ = D, d_ = d, D2 = D_ * D_, n = chi_ * D2;
  size_t need = 0;
  auto add = [&](size_t c) { need += ((c * 8 + 255) / 256) * 256; };
  add(chi_ * D2 * chi_);
  add(chi_ * D2 * D2 * chi_);
  add(chi_ * chi_ * d_ * D2 * D2);
  add(chi_ * chi_ * d_ * d_ * D2 * D2);
  add(chi_ * D2 * chi_);
  add(2 * chi_ * d_ * d_ * D2 * chi_);
  add(chi_ * D2 * chi_);
  add(3 * nsite * d_ * D2 * D2);
  TN_TRY(ws_reserve(ctx, need + (1 << 20)));
  ws_reset(ctx);
  Geo g;
  TN_TRY(setup_geo(ctx, g, Lx, Ly, D, d, nsite, sites, cell, chi, const_cast<double*>(C),
                   const_cast<double*>(T)));
  double* X1 = ws_alloc<double>(ctx, chi_ * D2 * chi_);
  double* X2 = ws_alloc<double>(ctx, chi_ * D2 * D2 * chi_);
  double* X3 = ws_alloc<double>(ctx, chi_ * chi_ * d_ * D2 * D2);
  double* X4 = ws_alloc<double>(ctx, chi_ * chi_ * d_ * d_ * D2 * D2);
  double* Y = ws_alloc<double>(ctx, chi_ * D2 * chi_);
  double* L1 = ws_alloc<double>(ctx, 2 * chi_ * d_ * d_ * D2 * chi_);
  double* L2 = L1 + chi_ * d_ * d_ * D2 * chi_;
  double* Rc = ws_alloc<double>(ctx, chi_ * D2 * chi_);
  if (!Rc) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted (rdms)");
  const long long cD = (long long)chi * D * D;
  const long long dd = d;
  for (int y = 0; y < Ly; ++y)
    for (int x = 0; x < Lx; ++x) {
      const int p = g.F.at(0, x, y);
      // one-site: L(0, p) closed by C2 T2 C3
      TN_TRY(half_left(ctx, g, 0, p, L1, X1, X2, X3, X4, Y));
      TN_TRY(gemm(ctx, chi, (int)(D2 * chi_), chi, g.Cp(p, 1), chi, false, g.Tp(p, 1),
                  (int)(D2 * chi_), false, X1, (int)(D2 * chi_), 1.0, 0.0));
      TN_TRY(gemm(ctx, (int)(chi_ * D2), chi, chi, X1, chi, false, g.Cp(p, 2), chi, false, Rc, chi,
                  1.0, 0.0));
      TN_TRY(tc_run(ctx, nets::rdm_one(chi, D, d), L1, Rc, rho1 + (long long)p * d * d, 1.0,
                    0.0));
      // horizontal pair (x, y)-(x+1, y): L(0, p) with L(2, q)
      const int q = g.F.at(0, x + 1, y);
      TN_TRY(half_left(ctx, g, 2, q, L2, X1, X2, X3, X4, Y));
      const Contraction c2 = nets::rdm_two(chi, D, d);
      TN_TRY(tc_run(ctx, c2, L1, L2, rhoh + (long long)p * d * d * d * d, 1.0, 0.0));
      // vertical pair: frame 1 (top site on the left) with frame 3 (bottom site)
      const int pb = g.F.at(0, x, y + 1);
      TN_TRY(half_left(ctx, g, 1, p, L1, X1, X2, X3, X4, Y));
      TN_TRY(half_left(ctx, g, 3, pb, L2, X1, X2, X3, X4, Y));
      TN_TRY(tc_run(ctx, c2, L1, L2, rhov + (long long)p * d * d * d * d, 1.0, 0.0));
    }
  (void)cD;
  const int npos = Lx * Ly;
  hipLaunchKernelGGL(trace_normalize_kernel, dim3(npos), dim3(64), 0, ctx->stream, rho1, d,
                     (long long)d * d);
  hipLaunchKernelGGL(trace_normalize_kernel, dim3(npos), dim3(64), 0, ctx->stream, rhoh, d * d,
                     (long long)d * d * d * d);
  hipLaunchKernelGGL(trace_normalize_kernel, dim3(npos), dim3(64), 0, ctx->stream, rhov, d * d,
                     (long long)d * d * d * d);
  TN_HIP(ctx, hipGetLastError());
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return TN_OK;
}
