// Reverse-mode derivative of the TFIM energy of a single-site iPEPS after a
// fixed number of CTMRG iterations (the energy function of the paper's 2D
// method, Sec. VI B and VI D, differentiated with respect to the site tensor).
//
// The forward pass is the directional CTMRG of the 1 x 1 cell written as a
// tape of primitive operations: table-driven contractions (adjoint: two more
// contractions), Frobenius normalisation, site rotation, trace
// normalisation, and the projector construction from the four enlarged
// corners.  For the projectors, K = (E2 E3)(E0 E1) is formed explicitly and
// given a full one-sided Jacobi SVD; the adjoint of the truncated SVD is the
// full-SVD formula restricted to the kept triplets, with the inverse gaps
// 1/g, g = s_j^2 - s_i^2, broadened to g/(g^2 + eps (s_i^2 + s_j^2)^2).
// Iterations are checkpointed every `ckpt` iterations: the forward pass keeps
// only the environments at the checkpoints, and the backward pass recomputes
// each segment with its tape before running it in reverse.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"
#include "nets.h"

namespace {

// ---------------------------------------------------------------------------
// device memory of one tape: 256-byte slices of 256 MiB chunks that the
// context keeps between calls (keyed by tag and index), so only the first
// call that needs a chunk allocates it
// ---------------------------------------------------------------------------
struct Pool {
  tn_ctx* ctx;
  const char* tag;
  size_t nchunk = 0, off = 0, cap = 0;
  char* cur = nullptr;
  Pool(tn_ctx* c, const char* t) : ctx(c), tag(t) {}
  double* alloc(size_t count) {
    const size_t bytes = ((count * sizeof(double) + 255) / 256) * 256;
    if (off + bytes > cap) {
      const size_t sz = std::max<size_t>(bytes, (size_t)256 << 20);
      void* p = nullptr;
      const std::string key = std::string("energy_grad:") + tag + ":" + std::to_string(nchunk);
      if (keep_buffer(ctx, key, sz, &p, nullptr) != TN_OK || !p) return nullptr;
      ++nchunk;
      cur = static_cast<char*>(p);
      off = 0;
      cap = sz;
    }
    double* r = reinterpret_cast<double*>(cur + off);
    off += bytes;
    return r;
  }
};

// ---------------------------------------------------------------------------
// kernels of the primitive operations and their adjoints
// ---------------------------------------------------------------------------
__device__ inline double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += red[i];
  return t;
}

// y = x / |x|_F, the norm kept for the adjoint
__global__ __launch_bounds__(1024) void norm_fwd_kernel(const double* __restrict__ x,
                                                        double* __restrict__ y, long long n,
                                                        double* __restrict__ nrm) {
  __shared__ double red[16];
  double a = 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) a += x[i] * x[i];
  const double s = sqrt(block_sum(a, red));
  if (threadIdx.x == 0) *nrm = s;
  const double inv = s > 0.0 ? 1.0 / s : 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) y[i] = x[i] * inv;
}

// dx += (dy - y <y, dy>) / |x|
__global__ __launch_bounds__(1024) void norm_bwd_kernel(const double* __restrict__ y,
                                                        const double* __restrict__ dy,
                                                        double* __restrict__ dx, long long n,
                                                        const double* __restrict__ nrm) {
  __shared__ double red[16];
  double a = 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) a += y[i] * dy[i];
  const double dot = block_sum(a, red);
  const double s = *nrm;
  const double inv = s > 0.0 ? 1.0 / s : 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) dx[i] += (dy[i] - y[i] * dot) * inv;
}

// one counter-clockwise rotation of a site tensor, new (l,r,d,u) = old (u,d,l,r):
// forward B[t] = A[src(t)], adjoint dA[src(t)] += dB[t] (a permutation)
__device__ inline long long rot_src(long long t, int D) {
  long long r = t;
  const int u2 = r % D;
  r /= D;
  const int d2 = r % D;
  r /= D;
  const int r2 = r % D;
  r /= D;
  const int l2 = r % D;
  r /= D;
  return (((r * D + d2) * D + u2) * D + r2) * D + l2;
}

__global__ void rot_fwd_kernel(const double* __restrict__ A, double* __restrict__ B, long long tot,
                               int D) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < tot) B[t] = A[rot_src(t, D)];
}

__global__ void rot_bwd_kernel(const double* __restrict__ dB, double* __restrict__ dA,
                               long long tot, int D) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < tot) dA[rot_src(t, D)] += dB[t];
}

// rho = X / tr X (dim x dim), the trace kept for the adjoint
__global__ void trnorm_fwd_kernel(const double* __restrict__ X, double* __restrict__ rho, int dim,
                                  double* __restrict__ tr) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double t = 0.0;
  for (int i = 0; i < dim; ++i) t += X[i * dim + i];
  *tr = t;
  for (int i = 0; i < dim * dim; ++i) rho[i] = X[i] / t;
}

// dX += (drho - I <drho, rho>) / tr
__global__ void trnorm_bwd_kernel(const double* __restrict__ rho, const double* __restrict__ drho,
                                  double* __restrict__ dX, int dim, const double* __restrict__ tr) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double dot = 0.0;
  for (int i = 0; i < dim * dim; ++i) dot += drho[i] * rho[i];
  const double t = *tr;
  for (int i = 0; i < dim; ++i)
    for (int j = 0; j < dim; ++j) dX[i * dim + j] += (drho[i * dim + j] - (i == j ? dot : 0.0)) / t;
}

// isq_j = s_j^-1/2 for s_j > 1e-14 s_0, else 0 (j < chi)
__global__ void isq_kernel(const double* __restrict__ s, double* __restrict__ isq, int chi, int n) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= chi) return;
  const double sj = j < n ? s[j] : 0.0;
  isq[j] = (j < n && sj > 1e-14 * s[0]) ? 1.0 / sqrt(sj) : 0.0;
}

// Y[i][j] = X[i][j] * isq[j], X with leading dimension ldx, Y n x chi
__global__ void scale_kept_kernel(const double* __restrict__ X, int ldx, const double* __restrict__ isq,
                                  double* __restrict__ Y, int n, int chi) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * chi) return;
  const int i = (int)(t / chi), j = (int)(t % chi);
  Y[t] = X[(long long)i * ldx + j] * isq[j];
}

// Adjoint inputs of the SVD from those of X = U_chi diag(isq), Y = V_chi diag(isq):
// Ub[:, j] = dX[:, j] isq_j, Vb likewise (n x n, zero beyond chi);
// Sb_j = -isq_j^3 / 2 * (sum_i U_ij dX_ij + V_ij dY_ij)
__global__ __launch_bounds__(256) void svd_bar_kernel(const double* __restrict__ U,
                                                      const double* __restrict__ V,
                                                      const double* __restrict__ dX,
                                                      const double* __restrict__ dY,
                                                      const double* __restrict__ isq, int n,
                                                      int chi, double* __restrict__ Ub,
                                                      double* __restrict__ Vb,
                                                      double* __restrict__ Sb) {
  const int j = blockIdx.x;  // column, < n
  __shared__ double red[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const long long e = (long long)i * n + j;
    if (j < chi) {
      const double dx = dX[(long long)i * chi + j], dy = dY[(long long)i * chi + j];
      Ub[e] = dx * isq[j];
      Vb[e] = dy * isq[j];
      acc += U[e] * dx + V[e] * dy;
    } else {
      Ub[e] = 0.0;
      Vb[e] = 0.0;
    }
  }
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) {
    const double q = j < chi ? isq[j] : 0.0;
    Sb[j] = -0.5 * q * q * q * tot;
  }
}

// M = (F o (Ju - Ju^T)) diag(s) + diag(Sb) + diag(s) (F o (Jv - Jv^T)),
// F_ij = g / (g^2 + eps (s_i^2 + s_j^2)^2), g = s_j^2 - s_i^2, for i != j
// (the broadening acts on the relative gap of the pair), F_ii = 0
__global__ void svd_mid_kernel(const double* __restrict__ Ju, const double* __restrict__ Jv,
                               const double* __restrict__ s, const double* __restrict__ Sb, int n,
                               double eps, double* __restrict__ M) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * n) return;
  const int i = (int)(t / n), j = (int)(t % n);
  if (i == j) {
    M[t] = Sb[i];
    return;
  }
  const double si2 = s[i] * s[i], sj2 = s[j] * s[j], g = sj2 - si2;
  const double den = g * g + eps * (si2 + sj2) * (si2 + sj2);
  const double F = den > 0.0 ? g / den : 0.0;
  const long long tt = (long long)j * n + i;
  M[t] = F * (Ju[t] - Ju[tt]) * s[j] + s[i] * F * (Jv[t] - Jv[tt]);
}

// ---------------------------------------------------------------------------
// the tape
// ---------------------------------------------------------------------------
enum OpKind { OP_TC, OP_NORM, OP_ROT, OP_TRNORM, OP_SVDPROJ };

struct Op {
  OpKind k;
  int prec = P_F64;  // precision of the products of this operation and of their adjoints
  Contraction c;
  int a = -1, b = -1, o = -1, o2 = -1;
  int e[4] = {-1, -1, -1, -1};
  int dim = 0;           // OP_TRNORM: matrix dimension; OP_ROT: D
  double* aux = nullptr;  // OP_NORM / OP_TRNORM: the norm or trace
  int sv = -1;           // OP_SVDPROJ: saved factorisation
};

struct SvdSave {
  int n, chi;
  double *Lft, *Rgt, *U, *S, *V, *isq;
};

struct Tape {
  tn_ctx* ctx;
  int prec;  // precision of the products recorded from now on
  double eps;
  Pool pool;
  std::vector<double*> v, g;
  std::vector<long long> len;
  std::vector<Op> ops;
  std::vector<SvdSave> svd;
  // factorisations of the forward pass, reused when a checkpoint segment is
  // recomputed: slot svd_slot holds U, V (n x n) and S (n) of one projector
  // problem; with svd_replay the slot is read instead of recomputed (the
  // recomputation is bitwise the forward pass: same inputs, same kernels)
  double* svd_cache = nullptr;
  int svd_slot = -1;
  bool svd_replay = false;

  explicit Tape(tn_ctx* c, int p, double e) : ctx(c), prec(p), eps(e), pool(c, "tape") {}

  int tensor(long long n) {
    double* p = pool.alloc((size_t)n);
    if (!p) return -1;
    v.push_back(p);
    g.push_back(nullptr);
    len.push_back(n);
    return (int)v.size() - 1;
  }
  double* scratch(long long n) { return pool.alloc((size_t)n); }
  // gradient buffer of tensor i, zeroed on first use
  double* grad(int i) {
    if (!g[i]) {
      g[i] = pool.alloc((size_t)len[i]);
      if (g[i]) (void)hipMemsetAsync(g[i], 0, len[i] * sizeof(double), ctx->stream);
    }
    return g[i];
  }
};

#define TP_NEW(id, tape, n)                                                       \
  const int id = (tape).tensor(n);                                                \
  if (id < 0) TN_FAIL((tape).ctx, TN_ENOMEM, "out of device memory in energy_grad")

// out = A (x) B
int t_tc(Tape& tp, const Contraction& c, int a, int b, long long out_len, int* out) {
  TP_NEW(o, tp, out_len);
  TN_TRY(tc_run(tp.ctx, c, tp.v[a], tp.v[b], tp.v[o], 1.0, 0.0, tp.prec));
  Op op;
  op.k = OP_TC;
  op.prec = tp.prec;
  op.c = c;
  op.a = a;
  op.b = b;
  op.o = o;
  tp.ops.push_back(op);
  *out = o;
  return TN_OK;
}

// C[M][N] = op(A) op(B), row-major leading dimensions
int t_mm(Tape& tp, int M, int N, int K, int a, long long lda, bool ta, int b, long long ldb,
         bool tb, int* out) {
  return t_tc(tp, nets::matmul(M, N, K, lda, ta, ldb, tb, N), a, b, (long long)M * N, out);
}

int t_norm(Tape& tp, int a, int* out) {
  TP_NEW(o, tp, tp.len[a]);
  double* nrm = tp.scratch(1);
  if (!nrm) TN_FAIL(tp.ctx, TN_ENOMEM, "out of device memory in energy_grad");
  hipLaunchKernelGGL(norm_fwd_kernel, dim3(1), dim3(1024), 0, tp.ctx->stream, tp.v[a], tp.v[o],
                     tp.len[a], nrm);
  TN_HIP(tp.ctx, hipGetLastError());
  Op op;
  op.k = OP_NORM;
  op.a = a;
  op.o = o;
  op.aux = nrm;
  tp.ops.push_back(op);
  *out = o;
  return TN_OK;
}

int t_rot(Tape& tp, int a, int D, int* out) {
  TP_NEW(o, tp, tp.len[a]);
  const long long tot = tp.len[a];
  hipLaunchKernelGGL(rot_fwd_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                     tp.ctx->stream, tp.v[a], tp.v[o], tot, D);
  TN_HIP(tp.ctx, hipGetLastError());
  Op op;
  op.k = OP_ROT;
  op.a = a;
  op.o = o;
  op.dim = D;
  tp.ops.push_back(op);
  *out = o;
  return TN_OK;
}

int t_trnorm(Tape& tp, int a, int dim, int* out) {
  TP_NEW(o, tp, tp.len[a]);
  double* tr = tp.scratch(1);
  if (!tr) TN_FAIL(tp.ctx, TN_ENOMEM, "out of device memory in energy_grad");
  hipLaunchKernelGGL(trnorm_fwd_kernel, dim3(1), dim3(1), 0, tp.ctx->stream, tp.v[a], tp.v[o], dim,
                     tr);
  TN_HIP(tp.ctx, hipGetLastError());
  Op op;
  op.k = OP_TRNORM;
  op.a = a;
  op.o = o;
  op.dim = dim;
  op.aux = tr;
  tp.ops.push_back(op);
  *out = o;
  return TN_OK;
}

// Projector pair of a row cut from its four enlarged corners (n x n each):
// K = (E2 E3)(E0 E1) = U S V^T, P = (E2 E3)^T U_chi S^-1/2,
// PtT = (E0 E1) V_chi S^-1/2 (singular values below 1e-14 s_1 dropped).
int t_svdproj(Tape& tp, const int e[4], int n, int chi, int* P, int* PtT) {
  tn_ctx* ctx = tp.ctx;
  SvdSave sv;
  sv.n = n;
  sv.chi = chi;
  const long long nn = (long long)n * n;
  const bool cached = tp.svd_cache && tp.svd_slot >= 0;
  const int slot_id = tp.svd_slot;
  tp.svd_slot = -1;  // one factorisation per slot
  sv.Lft = tp.scratch(nn);
  sv.Rgt = tp.scratch(nn);
  if (cached) {
    double* slot = tp.svd_cache + (size_t)slot_id * (size_t)(2 * nn + n);
    sv.U = slot;
    sv.V = slot + nn;
    sv.S = slot + 2 * nn;
  } else {
    sv.U = tp.scratch(nn);
    sv.V = tp.scratch(nn);
    sv.S = tp.scratch(n);
  }
  sv.isq = tp.scratch(chi);
  double* K = tp.scratch(nn);
  double* X = tp.scratch((long long)n * chi);
  if (!X) TN_FAIL(ctx, TN_ENOMEM, "out of device memory in energy_grad");
  TN_TRY(gemm(ctx, n, n, n, tp.v[e[2]], n, false, tp.v[e[3]], n, false, sv.Lft, n, 1.0, 0.0, 1, 0,
              0, 0, tp.prec));
  TN_TRY(gemm(ctx, n, n, n, tp.v[e[0]], n, false, tp.v[e[1]], n, false, sv.Rgt, n, 1.0, 0.0, 1, 0,
              0, 0, tp.prec));
  if (!(cached && tp.svd_replay)) {
    TN_TRY(gemm(ctx, n, n, n, sv.Lft, n, false, sv.Rgt, n, false, K, n, 1.0, 0.0, 1, 0, 0, 0,
                tp.prec));
    if (n > 128)
      TN_TRY(svd_qr_large(ctx, n, n, K, n, sv.U, n, sv.S, sv.V, n));
    else
      TN_TRY(jacobi_svd(ctx, 1, n, n, K, n, 0, sv.U, n, 0, sv.S, 0, sv.V, n, 0));
  }
  hipLaunchKernelGGL(isq_kernel, dim3((chi + 63) / 64), dim3(64), 0, ctx->stream, sv.S, sv.isq,
                     chi, n);
  TP_NEW(p, tp, (long long)n * chi);
  TP_NEW(pt, tp, (long long)n * chi);
  const unsigned gs = (unsigned)(((long long)n * chi + 255) / 256);
  hipLaunchKernelGGL(scale_kept_kernel, dim3(gs), dim3(256), 0, ctx->stream, sv.U, n, sv.isq, X, n,
                     chi);
  TN_TRY(gemm(ctx, n, chi, n, sv.Lft, n, true, X, chi, false, tp.v[p], chi, 1.0, 0.0, 1, 0, 0, 0,
              tp.prec));
  hipLaunchKernelGGL(scale_kept_kernel, dim3(gs), dim3(256), 0, ctx->stream, sv.V, n, sv.isq, X, n,
                     chi);
  TN_TRY(gemm(ctx, n, chi, n, sv.Rgt, n, false, X, chi, false, tp.v[pt], chi, 1.0, 0.0, 1, 0, 0,
              0, tp.prec));
  TN_HIP(ctx, hipGetLastError());
  tp.svd.push_back(sv);
  Op op;
  op.k = OP_SVDPROJ;
  op.prec = tp.prec;
  for (int j = 0; j < 4; ++j) op.e[j] = e[j];
  op.o = p;
  op.o2 = pt;
  op.sv = (int)tp.svd.size() - 1;
  tp.ops.push_back(op);
  *P = p;
  *PtT = pt;
  return TN_OK;
}

// adjoint of a contraction out = A (x) B: dA += dOut (x) B^T, dB += A^T (x) dOut
int b_tc(Tape& tp, const Op& op) {
  const Contraction& c = op.c;
  const double* dO = tp.g[op.o];
  Contraction ca;  // dA[m, k] = sum_n dOut[m, n] B[k, n]
  ca.am = c.cm;
  ca.ak = c.cn;
  ca.bk = c.bn;
  ca.bn = c.bk;
  ca.cm = c.am;
  ca.cn = c.ak;
  double* dA = tp.grad(op.a);
  if (!dA) TN_FAIL(tp.ctx, TN_ENOMEM, "out of device memory in energy_grad");
  TN_TRY(tc_run(tp.ctx, ca, dO, tp.v[op.b], dA, 1.0, 1.0, op.prec));
  Contraction cb;  // dB[k, n] = sum_m A[m, k] dOut[m, n]
  cb.am = c.ak;
  cb.ak = c.am;
  cb.bk = c.cm;
  cb.bn = c.cn;
  cb.cm = c.bk;
  cb.cn = c.bn;
  double* dB = tp.grad(op.b);
  if (!dB) TN_FAIL(tp.ctx, TN_ENOMEM, "out of device memory in energy_grad");
  TN_TRY(tc_run(tp.ctx, cb, tp.v[op.a], dO, dB, 1.0, 1.0, op.prec));
  return TN_OK;
}

int b_svdproj(Tape& tp, const Op& op) {
  tn_ctx* ctx = tp.ctx;
  const SvdSave& sv = tp.svd[op.sv];
  const int n = sv.n, chi = sv.chi;
  const long long nn = (long long)n * n, nc = (long long)n * chi;
  double* dP = tp.g[op.o];
  double* dPt = tp.g[op.o2];
  double* X = tp.scratch(nc);
  double* Y = tp.scratch(nc);
  double* dX = tp.scratch(nc);
  double* dY = tp.scratch(nc);
  double* dL = tp.scratch(nn);
  double* dR = tp.scratch(nn);
  double* Ub = tp.scratch(nn);
  double* Vb = tp.scratch(nn);
  double* Sb = tp.scratch(n);
  double* Ju = tp.scratch(nn);
  double* Jv = tp.scratch(nn);
  double* M = tp.scratch(nn);
  double* dK = tp.scratch(nn);
  if (!dK) TN_FAIL(ctx, TN_ENOMEM, "out of device memory in energy_grad");
  TN_HIP(ctx, hipMemsetAsync(dX, 0, nc * sizeof(double), ctx->stream));
  TN_HIP(ctx, hipMemsetAsync(dY, 0, nc * sizeof(double), ctx->stream));
  TN_HIP(ctx, hipMemsetAsync(dL, 0, nn * sizeof(double), ctx->stream));
  TN_HIP(ctx, hipMemsetAsync(dR, 0, nn * sizeof(double), ctx->stream));
  const unsigned gs = (unsigned)((nc + 255) / 256);
  hipLaunchKernelGGL(scale_kept_kernel, dim3(gs), dim3(256), 0, ctx->stream, sv.U, n, sv.isq, X, n,
                     chi);
  hipLaunchKernelGGL(scale_kept_kernel, dim3(gs), dim3(256), 0, ctx->stream, sv.V, n, sv.isq, Y, n,
                     chi);
  TN_HIP(ctx, hipGetLastError());
  // P = Lft^T X: dLft = X dP^T, dX = Lft dP
  if (dP) {
    TN_TRY(gemm(ctx, n, n, chi, X, chi, false, dP, chi, true, dL, n, 1.0, 0.0, 1, 0, 0, 0,
                op.prec));
    TN_TRY(gemm(ctx, n, chi, n, sv.Lft, n, false, dP, chi, false, dX, chi, 1.0, 0.0, 1, 0, 0, 0,
                op.prec));
  }
  // PtT = Rgt Y: dRgt = dPtT Y^T, dY = Rgt^T dPtT
  if (dPt) {
    TN_TRY(gemm(ctx, n, n, chi, dPt, chi, false, Y, chi, true, dR, n, 1.0, 0.0, 1, 0, 0, 0,
                op.prec));
    TN_TRY(gemm(ctx, n, chi, n, sv.Rgt, n, true, dPt, chi, false, dY, chi, 1.0, 0.0, 1, 0, 0, 0,
                op.prec));
  }
  // SVD adjoint (FP64): dK = U M V^T
  hipLaunchKernelGGL(svd_bar_kernel, dim3(n), dim3(256), 0, ctx->stream, sv.U, sv.V, dX, dY,
                     sv.isq, n, chi, Ub, Vb, Sb);
  TN_HIP(ctx, hipGetLastError());
  TN_TRY(gemm(ctx, n, n, n, sv.U, n, true, Ub, n, false, Ju, n, 1.0, 0.0));
  TN_TRY(gemm(ctx, n, n, n, sv.V, n, true, Vb, n, false, Jv, n, 1.0, 0.0));
  hipLaunchKernelGGL(svd_mid_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0,
                     ctx->stream, Ju, Jv, sv.S, Sb, n, tp.eps, M);
  TN_HIP(ctx, hipGetLastError());
  TN_TRY(gemm(ctx, n, n, n, sv.U, n, false, M, n, false, Ju, n, 1.0, 0.0));
  TN_TRY(gemm(ctx, n, n, n, Ju, n, false, sv.V, n, true, dK, n, 1.0, 0.0));
  // K = Lft Rgt
  TN_TRY(gemm(ctx, n, n, n, dK, n, false, sv.Rgt, n, true, dL, n, 1.0, 1.0, 1, 0, 0, 0, op.prec));
  TN_TRY(gemm(ctx, n, n, n, sv.Lft, n, true, dK, n, false, dR, n, 1.0, 1.0, 1, 0, 0, 0, op.prec));
  // Lft = E2 E3, Rgt = E0 E1
  double* g0 = tp.grad(op.e[0]);
  double* g1 = tp.grad(op.e[1]);
  double* g2 = tp.grad(op.e[2]);
  double* g3 = tp.grad(op.e[3]);
  if (!g0 || !g1 || !g2 || !g3) TN_FAIL(ctx, TN_ENOMEM, "out of device memory in energy_grad");
  TN_TRY(gemm(ctx, n, n, n, dL, n, false, tp.v[op.e[3]], n, true, g2, n, 1.0, 1.0, 1, 0, 0, 0,
              op.prec));
  TN_TRY(gemm(ctx, n, n, n, tp.v[op.e[2]], n, true, dL, n, false, g3, n, 1.0, 1.0, 1, 0, 0, 0,
              op.prec));
  TN_TRY(gemm(ctx, n, n, n, dR, n, false, tp.v[op.e[1]], n, true, g0, n, 1.0, 1.0, 1, 0, 0, 0,
              op.prec));
  TN_TRY(gemm(ctx, n, n, n, tp.v[op.e[0]], n, true, dR, n, false, g1, n, 1.0, 1.0, 1, 0, 0, 0,
              op.prec));
  return TN_OK;
}

// Run the tape backwards from the gradients already seeded on its outputs.
int backward(Tape& tp) {
  tn_ctx* ctx = tp.ctx;
  for (int i = (int)tp.ops.size() - 1; i >= 0; --i) {
    const Op& op = tp.ops[i];
    const bool live = tp.g[op.o] || (op.o2 >= 0 && tp.g[op.o2]);
    if (!live) continue;
    switch (op.k) {
      case OP_TC:
        TN_TRY(b_tc(tp, op));
        break;
      case OP_NORM: {
        double* dx = tp.grad(op.a);
        if (!dx) TN_FAIL(ctx, TN_ENOMEM, "out of device memory in energy_grad");
        hipLaunchKernelGGL(norm_bwd_kernel, dim3(1), dim3(1024), 0, ctx->stream, tp.v[op.o],
                           tp.g[op.o], dx, tp.len[op.o], op.aux);
        break;
      }
      case OP_ROT: {
        double* dx = tp.grad(op.a);
        if (!dx) TN_FAIL(ctx, TN_ENOMEM, "out of device memory in energy_grad");
        const long long tot = tp.len[op.o];
        hipLaunchKernelGGL(rot_bwd_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                           ctx->stream, tp.g[op.o], dx, tot, op.dim);
        break;
      }
      case OP_TRNORM: {
        double* dx = tp.grad(op.a);
        if (!dx) TN_FAIL(ctx, TN_ENOMEM, "out of device memory in energy_grad");
        hipLaunchKernelGGL(trnorm_bwd_kernel, dim3(1), dim3(1), 0, ctx->stream, tp.v[op.o],
                           tp.g[op.o], dx, op.dim, op.aux);
        break;
      }
      case OP_SVDPROJ:
        TN_TRY(b_svdproj(tp, op));
        break;
    }
    TN_HIP(ctx, hipGetLastError());
  }
  return TN_OK;
}

// ---------------------------------------------------------------------------
// the 1 x 1 cell: environment slots k = 0..3 (C1..C4, T1..T4), site rotated
// by f in frame f; one CTMRG iteration is the left move in frames 0..3
// ---------------------------------------------------------------------------
struct Env {
  int C[4], T[4];
};

struct Shape {
  int chi, D, d, n;
  long long csz() const { return (long long)chi * chi; }
  long long tsz() const { return (long long)chi * D * D * chi; }
};

// Enlarged upper-left corner of frame f: E[(a, dk, db), (b, rk, rb)]
int t_corner(Tape& tp, const Shape& s, const Env& env, const int* arot, int f, int* E) {
  const long long chi = s.chi, D = s.D, D2 = D * D;
  const int c = env.C[f & 3], t1 = env.T[f & 3], t4 = env.T[(f + 3) & 3], a = arot[f & 3];
  int x1, x2, x3;
  TN_TRY(t_mm(tp, (int)(chi * D2), (int)chi, (int)chi, t4, chi, false, c, chi, false, &x1));
  TN_TRY(t_mm(tp, (int)(chi * D2), (int)(D2 * chi), (int)chi, x1, chi, false, t1, D2 * chi, false,
              &x2));
  TN_TRY(t_tc(tp, nets::corner_ket(chi, D, s.d), x2, a, chi * chi * s.d * D2 * D2, &x3));
  TN_TRY(t_tc(tp, nets::corner_bra(chi, D, s.d, s.n), x3, a, (long long)s.n * s.n, E));
  return TN_OK;
}

// left move in frame f (the 1 x 1 cell has one column and one row cut)
int t_move(Tape& tp, const Shape& s, Env& env, const int* arot, int f) {
  const long long chi = s.chi, D = s.D, D2 = D * D, n = s.n;
  int E[4];
  for (int j = 0; j < 4; ++j) TN_TRY(t_corner(tp, s, env, arot, f + j, &E[j]));
  int P, PtT;
  TN_TRY(t_svdproj(tp, E, (int)n, (int)chi, &P, &PtT));
  const int c1 = env.C[f & 3], t1 = env.T[f & 3], t3 = env.T[(f + 2) & 3];
  const int c4 = env.C[(f + 3) & 3], t4 = env.T[(f + 3) & 3], a = arot[f & 3];
  // C1' = P^T (C1 T1)
  int ct, cn1;
  TN_TRY(t_mm(tp, (int)chi, (int)(D2 * chi), (int)chi, c1, chi, false, t1, D2 * chi, false, &ct));
  TN_TRY(t_mm(tp, (int)chi, (int)chi, (int)n, P, chi, true, ct, chi, false, &cn1));
  // C4' = (T3 C4) PtT
  int z, cn4;
  TN_TRY(t_tc(tp, nets::t3_c4(chi, D, n), t3, c4, chi * n, &z));
  TN_TRY(t_mm(tp, (int)chi, (int)chi, (int)n, z, n, false, PtT, chi, false, &cn4));
  // T4' = Pt (T4 a a) P
  int y1, y2, y3, tn4;
  TN_TRY(t_tc(tp, nets::edge_pt(chi, D, n), PtT, t4, chi * D2 * n, &y1));
  TN_TRY(t_tc(tp, nets::edge_ket(chi, D, s.d, n), y1, a, chi * chi * s.d * D2 * D2, &y2));
  TN_TRY(t_tc(tp, nets::edge_bra(chi, D, s.d, n), y2, a, chi * D2 * n, &y3));
  TN_TRY(t_tc(tp, nets::edge_p(chi, D, n), y3, P, s.tsz(), &tn4));
  int nc1, nt4, nc4;
  TN_TRY(t_norm(tp, cn1, &nc1));
  TN_TRY(t_norm(tp, tn4, &nt4));
  TN_TRY(t_norm(tp, cn4, &nc4));
  env.C[f & 3] = nc1;
  env.T[(f + 3) & 3] = nt4;
  env.C[(f + 3) & 3] = nc4;
  return TN_OK;
}

// half network of the RDMs in frame f: L[t, s, s', rk, rb, b]
int t_half(Tape& tp, const Shape& s, const Env& env, const int* arot, int f, int* L) {
  const long long chi = s.chi, D = s.D, D2 = D * D, n = s.n, d = s.d;
  const int c1 = env.C[f & 3], t1 = env.T[f & 3], t4 = env.T[(f + 3) & 3];
  const int c4 = env.C[(f + 3) & 3], t3 = env.T[(f + 2) & 3], a = arot[f & 3];
  int x1, x2, x3, x4, y;
  TN_TRY(t_mm(tp, (int)(chi * D2), (int)chi, (int)chi, t4, chi, false, c1, chi, false, &x1));
  TN_TRY(t_mm(tp, (int)(chi * D2), (int)(D2 * chi), (int)chi, x1, chi, false, t1, D2 * chi, false,
              &x2));
  TN_TRY(t_tc(tp, nets::corner_ket(chi, D, d), x2, a, chi * chi * d * D2 * D2, &x3));
  TN_TRY(t_tc(tp, nets::half_bra(chi, D, d, n), x3, a, chi * chi * d * d * D2 * D2, &x4));
  TN_TRY(t_mm(tp, (int)(chi * D2), (int)chi, (int)chi, t3, chi, false, c4, chi, false, &y));
  TN_TRY(t_tc(tp, nets::half_close(chi, D, d, n), x4, y, chi * d * d * D2 * chi, L));
  return TN_OK;
}

// reduced density matrices of the 1 x 1 cell (one site, horizontal and
// vertical pairs), each trace-normalised
int t_rdms(Tape& tp, const Shape& s, const Env& env, const int* arot, int* r1, int* rh, int* rv) {
  const long long chi = s.chi, D = s.D, D2 = D * D, d = s.d;
  int l0, l2, l1, l3, x1, rc, q1, qh, qv;
  TN_TRY(t_half(tp, s, env, arot, 0, &l0));
  TN_TRY(t_mm(tp, (int)chi, (int)(D2 * chi), (int)chi, env.C[1], chi, false, env.T[1], D2 * chi,
              false, &x1));
  TN_TRY(t_mm(tp, (int)(chi * D2), (int)chi, (int)chi, x1, chi, false, env.C[2], chi, false, &rc));
  TN_TRY(t_tc(tp, nets::rdm_one(chi, D, d), l0, rc, d * d, &q1));
  TN_TRY(t_half(tp, s, env, arot, 2, &l2));
  TN_TRY(t_tc(tp, nets::rdm_two(chi, D, d), l0, l2, d * d * d * d, &qh));
  TN_TRY(t_half(tp, s, env, arot, 1, &l1));
  TN_TRY(t_half(tp, s, env, arot, 3, &l3));
  TN_TRY(t_tc(tp, nets::rdm_two(chi, D, d), l1, l3, d * d * d * d, &qv));
  TN_TRY(t_trnorm(tp, q1, (int)d, r1));
  TN_TRY(t_trnorm(tp, qh, (int)(d * d), rh));
  TN_TRY(t_trnorm(tp, qv, (int)(d * d), rv));
  return TN_OK;
}

// tape inputs: the site (and its rotations) and the environment of a state
int t_inputs(Tape& tp, const Shape& s, const double* A, const double* C, const double* T,
             int* a_id, int arot[4], Env& env) {
  tn_ctx* ctx = tp.ctx;
  const long long asz = (long long)s.d * s.D * s.D * s.D * s.D;
  TP_NEW(a, tp, asz);
  TN_HIP(ctx, hipMemcpyAsync(tp.v[a], A, asz * sizeof(double), hipMemcpyDeviceToDevice,
                             ctx->stream));
  arot[0] = a;
  for (int f = 1; f < 4; ++f) TN_TRY(t_rot(tp, arot[f - 1], s.D, &arot[f]));
  for (int k = 0; k < 4; ++k) {
    TP_NEW(c, tp, s.csz());
    TP_NEW(t, tp, s.tsz());
    TN_HIP(ctx, hipMemcpyAsync(tp.v[c], C + k * s.csz(), s.csz() * sizeof(double),
                               hipMemcpyDeviceToDevice, ctx->stream));
    TN_HIP(ctx, hipMemcpyAsync(tp.v[t], T + k * s.tsz(), s.tsz() * sizeof(double),
                               hipMemcpyDeviceToDevice, ctx->stream));
    env.C[k] = c;
    env.T[k] = t;
  }
  *a_id = a;
  return TN_OK;
}

int copy_env_out(Tape& tp, const Shape& s, const Env& env, double* C, double* T) {
  for (int k = 0; k < 4; ++k) {
    TN_HIP(tp.ctx, hipMemcpyAsync(C + k * s.csz(), tp.v[env.C[k]], s.csz() * sizeof(double),
                                  hipMemcpyDeviceToDevice, tp.ctx->stream));
    TN_HIP(tp.ctx, hipMemcpyAsync(T + k * s.tsz(), tp.v[env.T[k]], s.tsz() * sizeof(double),
                                  hipMemcpyDeviceToDevice, tp.ctx->stream));
  }
  return TN_OK;
}

__global__ void axpy_kernel(const double* __restrict__ x, double* __restrict__ y, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += x[i];
}

int add_into(tn_ctx* ctx, const double* x, double* y, long long n) {
  hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream, x,
                     y, n);
  TN_HIP(ctx, hipGetLastError());
  return TN_OK;
}

// Gradients of a tape's inputs after its backward pass: the site (its
// rotations flow back into it) and the environment, added into dA, dC, dT.
int gather_input_grads(Tape& tp, const Shape& s, int a_id, const Env& env0, double* dA, double* dC,
                       double* dT) {
  const long long asz = (long long)s.d * s.D * s.D * s.D * s.D;
  if (tp.g[a_id]) TN_TRY(add_into(tp.ctx, tp.g[a_id], dA, asz));
  for (int k = 0; k < 4; ++k) {
    if (dC && tp.g[env0.C[k]]) TN_TRY(add_into(tp.ctx, tp.g[env0.C[k]], dC + k * s.csz(), s.csz()));
    if (dT && tp.g[env0.T[k]]) TN_TRY(add_into(tp.ctx, tp.g[env0.T[k]], dT + k * s.tsz(), s.tsz()));
  }
  return TN_OK;
}

// seed the gradients of a tape's output environment
int seed_env(Tape& tp, const Shape& s, const Env& env, const double* dC, const double* dT) {
  for (int k = 0; k < 4; ++k) {
    double* gc = tp.grad(env.C[k]);
    double* gt = tp.grad(env.T[k]);
    if (!gc || !gt) TN_FAIL(tp.ctx, TN_ENOMEM, "out of device memory in energy_grad");
    TN_TRY(add_into(tp.ctx, dC + k * s.csz(), gc, s.csz()));
    TN_TRY(add_into(tp.ctx, dT + k * s.tsz(), gt, s.tsz()));
  }
  return TN_OK;
}

}  // namespace

int energy_grad_impl(tn_ctx* ctx, int D, int d, double J, double h, const double* A, int chi,
                     const double* C0, const double* T0, int n_iter, int ckpt, int prec, double eps,
                     double* energy, double* dEdA) {
  if (!A || !C0 || !T0 || !energy || !dEdA) TN_FAIL(ctx, TN_EINVAL, "null pointer argument");
  if (d != 2) TN_FAIL(ctx, TN_EINVAL, "energy_grad is the TFIM energy: d must be 2");
  if (D < 1 || chi < 1) TN_FAIL(ctx, TN_EINVAL, "bad bond dimensions (D=%d chi=%d)", D, chi);
  if (n_iter < 0 || ckpt < 1) TN_FAIL(ctx, TN_EINVAL, "bad iteration count or checkpoint interval");
  // FP32 bulk contractions make E(A) after a fixed number of iterations from
  // a random boundary an ill-conditioned function: the rounding of the early
  // iterations decides which small singular values of the projector problems
  // come close, and the inverse gaps of the SVD adjoint amplify that, so its
  // gradient has no bound to state
  if (prec != P_F64)
    TN_FAIL(ctx, TN_EINVAL, "energy_grad runs in FP64 only (precision %d given)", prec);
  if (!(eps >= 0.0)) TN_FAIL(ctx, TN_EINVAL, "broadening must be >= 0");
  Shape s;
  s.chi = chi;
  s.D = D;
  s.d = d;
  s.n = chi * D * D;
  if (s.n > 512) TN_FAIL(ctx, TN_EINVAL, "energy_grad needs chi D^2 <= 512 (got %d)", s.n);
  const long long asz = (long long)d * D * D * D * D, ce = 4 * s.csz(), te = 4 * s.tsz();
  // checkpoints: environments at iterations 0, ckpt, 2 ckpt, ... (< n_iter)
  const int nck = n_iter == 0 ? 1 : (n_iter + ckpt - 1) / ckpt;
  // FP32 bulk: the last n_polish iterations and the energy run in FP64, as the
  // polish iterations of the CTMRG precision form
  const int n_polish = std::min(n_iter, 5);
  auto it_prec = [&](int it) { return it >= n_iter - n_polish ? (int)P_F64 : prec; };
  Pool keep(ctx, "keep");
  double* ck = keep.alloc((size_t)nck * (ce + te));
  double* cur = keep.alloc((size_t)(ce + te));
  double* gC = keep.alloc((size_t)ce);
  double* gT = keep.alloc((size_t)te);
  double* gC2 = keep.alloc((size_t)ce);
  double* gT2 = keep.alloc((size_t)te);
  if (!ck || !cur || !gC2 || !gT2) TN_FAIL(ctx, TN_ENOMEM, "out of device memory in energy_grad");
  // the forward pass's projector factorisations (one per move), reused by
  // the recomputation of the checkpoint segments; without the memory the
  // segments recompute them
  Pool svd_pool(ctx, "svd");
  const size_t svd_per = 2 * (size_t)s.n * s.n + s.n;
  double* svd_cache = n_iter > 0 ? svd_pool.alloc((size_t)n_iter * 4 * svd_per) : nullptr;
  if (!svd_cache) ctx->err.clear();
  TN_HIP(ctx, hipMemcpyAsync(cur, C0, ce * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  TN_HIP(ctx, hipMemcpyAsync(cur + ce, T0, te * sizeof(double), hipMemcpyDeviceToDevice,
                             ctx->stream));
  TN_HIP(ctx, hipMemsetAsync(dEdA, 0, asz * sizeof(double), ctx->stream));
  // forward pass, keeping the checkpoints
  for (int it = 0; it < n_iter; ++it) {
    if (it % ckpt == 0)
      TN_HIP(ctx, hipMemcpyAsync(ck + (size_t)(it / ckpt) * (ce + te), cur,
                                 (ce + te) * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    Tape tp(ctx, it_prec(it), eps);
    tp.svd_cache = svd_cache;
    int a_id, arot[4];
    Env env;
    TN_TRY(t_inputs(tp, s, A, cur, cur + ce, &a_id, arot, env));
    for (int f = 0; f < 4; ++f) {
      tp.svd_slot = 4 * it + f;
      TN_TRY(t_move(tp, s, env, arot, f));
    }
    TN_TRY(copy_env_out(tp, s, env, cur, cur + ce));
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  }
  if (n_iter == 0)
    TN_HIP(ctx, hipMemcpyAsync(ck, cur, (ce + te) * sizeof(double), hipMemcpyDeviceToDevice,
                               ctx->stream));
  // energy and its adjoint
  {
    Tape tp(ctx, P_F64, eps);
    int a_id, arot[4], r1, rh, rv;
    Env env;
    TN_TRY(t_inputs(tp, s, A, cur, cur + ce, &a_id, arot, env));
    TN_TRY(t_rdms(tp, s, env, arot, &r1, &rh, &rv));
    double hr[4 + 16 + 16];
    TN_HIP(ctx, hipMemcpyAsync(hr, tp.v[r1], 4 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    TN_HIP(ctx, hipMemcpyAsync(hr + 4, tp.v[rh], 16 * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
    TN_HIP(ctx, hipMemcpyAsync(hr + 20, tp.v[rv], 16 * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
    // E = -J <zz>_h - J <zz>_v - h <x>; dE/drho = the operators (symmetric)
    const double zz[4] = {1.0, -1.0, -1.0, 1.0};
    double e = -h * (hr[1] + hr[2]);
    double s1[4] = {0.0, -h, -h, 0.0}, sh[16], sv[16];
    for (int i = 0; i < 16; ++i) {
      sh[i] = 0.0;
      sv[i] = 0.0;
    }
    for (int i = 0; i < 4; ++i) {
      e += -J * zz[i] * (hr[4 + 5 * i] + hr[20 + 5 * i]);
      sh[5 * i] = -J * zz[i];
      sv[5 * i] = -J * zz[i];
    }
    *energy = e;
    if (!std::isfinite(e)) TN_FAIL(ctx, TN_ENUMERIC, "non-finite energy");
    double* g1 = tp.grad(r1);
    double* gh = tp.grad(rh);
    double* gv = tp.grad(rv);
    if (!g1 || !gh || !gv) TN_FAIL(ctx, TN_ENOMEM, "out of device memory in energy_grad");
    TN_HIP(ctx, hipMemcpyAsync(g1, s1, 4 * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    TN_HIP(ctx, hipMemcpyAsync(gh, sh, 16 * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    TN_HIP(ctx, hipMemcpyAsync(gv, sv, 16 * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    TN_TRY(backward(tp));
    TN_HIP(ctx, hipMemsetAsync(gC, 0, ce * sizeof(double), ctx->stream));
    TN_HIP(ctx, hipMemsetAsync(gT, 0, te * sizeof(double), ctx->stream));
    TN_TRY(gather_input_grads(tp, s, a_id, env, dEdA, gC, gT));
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  }
  // segments in reverse: recompute with the tape, then run it backwards
  for (int sg = (n_iter == 0 ? -1 : nck - 1); sg >= 0; --sg) {
    const int i0 = sg * ckpt, i1 = std::min(n_iter, i0 + ckpt);
    Tape tp(ctx, prec, eps);
    int a_id, arot[4];
    Env env0, env;
    const double* cs = ck + (size_t)sg * (ce + te);
    TN_TRY(t_inputs(tp, s, A, cs, cs + ce, &a_id, arot, env0));
    env = env0;
    tp.svd_cache = svd_cache;
    tp.svd_replay = true;
    for (int it = i0; it < i1; ++it) {
      tp.prec = it_prec(it);
      for (int f = 0; f < 4; ++f) {
        tp.svd_slot = 4 * it + f;
        TN_TRY(t_move(tp, s, env, arot, f));
      }
    }
    TN_TRY(seed_env(tp, s, env, gC, gT));
    TN_TRY(backward(tp));
    TN_HIP(ctx, hipMemsetAsync(gC2, 0, ce * sizeof(double), ctx->stream));
    TN_HIP(ctx, hipMemsetAsync(gT2, 0, te * sizeof(double), ctx->stream));
    TN_TRY(gather_input_grads(tp, s, a_id, env0, dEdA, gC2, gT2));
    std::swap(gC, gC2);
    std::swap(gT, gT2);
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  }
  return TN_OK;
}
