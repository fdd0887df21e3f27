// Shared host-side definitions for the HIP library: context, workspace arena,
// offset-table cache and error handling.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "itebd.h"

// Capacity in doubles of the context's pinned host staging buffer; every
// read-back into it checks its extent against this.
constexpr size_t TN_HOST_SCRATCH = 1024;

struct tn_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  std::string err;
  // bump arena for per-call scratch
  char* arena = nullptr;
  size_t arena_size = 0;
  size_t arena_off = 0;
  // persistent device allocations: offset tables keyed by their description
  std::map<std::string, int*> tables;
  // persistent per-key device buffers (warm starts of iterative solvers)
  std::map<std::string, std::pair<void*, size_t>> keep;
  std::map<std::string, std::vector<char>> keep_flags;  // host validity flags per buffer slot
  // pinned host staging for small scalar read-backs (TN_HOST_SCRATCH doubles)
  double* host_scratch = nullptr;
  // a second stream of the library's own (default priority) for work that
  // overlaps the context stream; forked from it and joined back by events
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // optional per-launch timing of the contraction kernel (HIP events on the
  // context stream) and the algorithmic flops of each timed launch
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<double> prof_flops;
  double prof_bytes = 0.0;  // algorithmic bytes of the timed contractions
  // solver counters since the last read
  long long svd_iters = 0, svd_calls = 0, svd_unconverged = 0, svd_explicit = 0, moves = 0;
};

#define TN_FAIL(ctx, code, ...)                                   \
  do {                                                            \
    char _b[512];                                                 \
    snprintf(_b, sizeof(_b), __VA_ARGS__);                        \
    (ctx)->err = _b;                                              \
    return (code);                                                \
  } while (0)

#define TN_HIP(ctx, call)                                                    \
  do {                                                                       \
    hipError_t _e = (call);                                                  \
    if (_e != hipSuccess)                                                    \
      TN_FAIL(ctx, TN_EHIP, "%s failed: %s (%s:%d)", #call,                  \
              hipGetErrorString(_e), __FILE__, __LINE__);                   \
  } while (0)

#define TN_TRY(expr)            \
  do {                          \
    int _rc = (expr);           \
    if (_rc < 0) return _rc;    \
  } while (0)

// Arena: reserve grows the arena to at least `bytes` (only between uses);
// alloc hands out 256-byte aligned slices until reset.
int ws_reserve(tn_ctx* ctx, size_t bytes);
void* ws_alloc_bytes(tn_ctx* ctx, size_t bytes);
template <class T>
T* ws_alloc(tn_ctx* ctx, size_t count) {
  return static_cast<T*>(ws_alloc_bytes(ctx, count * sizeof(T)));
}
inline void ws_reset(tn_ctx* ctx) { ctx->arena_off = 0; }

// Persistent buffer keyed by name; (re)allocated when the size changes.
// `fresh` is set when the buffer was just created.
int keep_buffer(tn_ctx* ctx, const std::string& key, size_t bytes, void** ptr, bool* fresh);

// ---------------------------------------------------------------------------
// index groups and table-driven contractions
// ---------------------------------------------------------------------------

// One group of indices of an operand: extents and element strides, the last
// index fastest.  The flat index of the group runs over the product of the
// extents in row-major order.
struct IdxGroup {
  std::vector<int> ext;
  std::vector<long long> str;
  long long size() const {
    long long s = 1;
    for (int e : ext) s *= e;
    return s;
  }
};

inline IdxGroup grp(std::initializer_list<std::pair<int, long long>> l) {
  IdxGroup g;
  for (auto& p : l) {
    g.ext.push_back(p.first);
    g.str.push_back(p.second);
  }
  return g;
}

enum Prec { P_F64 = 0, P_F32 = 1, P_BF16 = 2 };

// C[c0 + cm(m) + cn(n)] = alpha * sum_k A[a0 + am(m) + ak(k)] * B[b0 + bk(k) + bn(n)]
//                         + beta * C[...]
// for a batch of `batch` problems with element strides sa, sb, sc.
// All pointers are device pointers to double.
struct Contraction {
  IdxGroup am, ak, bk, bn, cm, cn;
  int batch = 1;
  long long sa = 0, sb = 0, sc = 0;
};

int tc_run(tn_ctx* ctx, const Contraction& c, const double* A, const double* B, double* C,
           double alpha, double beta, int prec = P_F64);

// Pairwise contraction by index labels ("xlLg,gh->xlLh"): labels shared by
// A and B and absent from the output are summed; every output label comes
// from exactly one operand; all operands row-major with the given extents.
int ein(tn_ctx* ctx, const char* spec, const double* A, std::initializer_list<int> da,
        const double* B, std::initializer_list<int> db, double* C, double alpha = 1.0,
        double beta = 0.0, int prec = P_F64);

// Plain strided GEMM helper (row-major storage with leading dimensions;
// ta/tb transpose the stored operand).
int gemm(tn_ctx* ctx, int M, int N, int K, const double* A, int lda, bool ta, const double* B,
         int ldb, bool tb, double* C, int ldc, double alpha, double beta, int batch = 1,
         long long sa = 0, long long sb = 0, long long sc = 0, int prec = P_F64);

// ---------------------------------------------------------------------------
// small dense linear algebra on the device (FP64)
// ---------------------------------------------------------------------------

// Batched one-sided Jacobi SVD of m x n matrices (m >= n) stored row-major
// with leading dimension lda; A is overwritten.  Outputs U (m x n, row-major
// ldu), S (n, descending) and V (n x n, row-major ldv); each column of U is
// sign-fixed so that its largest-magnitude entry is positive.  Any output
// pointer may be null.  `sweeps` (device int per batch entry, may be null)
// returns the sweep count.
int jacobi_svd(tn_ctx* ctx, int batch, int m, int n, double* A, int lda, long long sA, double* U,
               int ldu, long long sU, double* S, long long sS, double* V, int ldv, long long sV);

// Whether jacobi_svd of these sizes takes workspace from the arena (else it
// runs in LDS alone).
bool jacobi_svd_needs_workspace(int m, int n);

// The side stream and its fork / join events, created on first use.
int side_stream_ready(tn_ctx* ctx);

// The same SVD for one matrix with n <= 512, spread over the whole GPU (one
// launch per round of column pairs, one workgroup per pair).  A is not
// modified; U m x n, S n, V n x n as for jacobi_svd.
int jacobi_svd_large(tn_ctx* ctx, int m, int n, const double* A, int lda, double* U, int ldu,
                     double* S, double* V, int ldv);
// the same factorisation with a Householder QR preconditioner (Jacobi on R^T)
int svd_qr_large(tn_ctx* ctx, int m, int n, const double* A, int lda, double* U, int ldu,
                 double* S, double* V, int ldv);

// Upper Cholesky factor of (G + shift*I) and its inverse, k x k row-major, for
// `batch` matrices stored back to back (info: one int per matrix, 0 or the
// failing pivot + 1).  The shift is shift_rel times the trace of G.
int cholesky_inv(tn_ctx* ctx, int k, const double* G, double shift_rel, double* R, double* Rinv,
                 int* info, int batch = 1);

// Misc kernels.
int scale_columns(tn_ctx* ctx, int m, int n, double* X, int ldx, const double* s, int invsqrt);
int frob_normalize(tn_ctx* ctx, double* x, long long n, double* norm_out);
// dst = src / ||src||_F (dst may be src; a zero tensor is copied as is)
int frob_normalize_to(tn_ctx* ctx, const double* src, double* dst, long long n,
                      double* norm_out);
int fill_random(tn_ctx* ctx, double* x, long long n, unsigned long long seed);
