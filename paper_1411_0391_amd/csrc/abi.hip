// C ABI entry points and context management.
#include <cmath>
#include <cstring>

#include "common.h"

int ctmrg_run_impl(tn_ctx* ctx, int Lx, int Ly, int D, int d, int nsite, const double* sites,
                   const int* cell, int chi, double* C, double* T, int max_iter, double tol,
                   int n_moves, int first_dir, int* iters, double* delta, int prec,
                   int n_polish);
int ipeps_rdms_impl(tn_ctx* ctx, int Lx, int Ly, int D, int d, int nsite, const double* sites,
                    const int* cell, int chi, const double* C, const double* T, double* rho1,
                    double* rhoh, double* rhov);

int jacobi_sweeps_read(tn_ctx* ctx, unsigned long long* out);
size_t env1d_doubles(int chi, int d);
int tm_fixed_point_impl(tn_ctx* ctx, int n_sites, int chi, int d, const double* ket,
                        const double* bra, double* vl, double* vr, double* eta, double tol,
                        int max_iter, int* iters, int flags);
int tm_fixed_point_noalloc_impl(tn_ctx* ctx, int n_sites, int chi, int d, const double* ket,
                                const double* bra, double* vl, double* vr, double* eta,
                                double tol, int max_iter, int* iters, int flags);
int noalloc_scratch_init(int device);
int itebd_step_impl(tn_ctx* ctx, int chi, int d, double* A, double J, double h, double dt, int mode,
                    double* env1d, double* lambda_out, double tol, double* trunc_err,
                    double* energy_or_null);
int ising2d_tm_step_impl(tn_ctx* ctx, int chi, double* A, double beta, int mode, double* env1d,
                         double* lambda_out, double tol, double* trunc_err, double* lnz_or_null);

int cell_links_impl(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, int* nlink,
                    int* links);
int ipeps_gate_impl(tn_ctx* ctx, int nsite, int D, int d, double J, double h, double dt,
                    const double* A, double* Theta);
int ipeps_truncate_impl(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, int d, int Din,
                        int Dout, const double* Theta, const double* P, const double* Q,
                        double* Aout);
int ipeps_canonicalize_impl(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, int d, int D,
                            int Dkeep, const double* A, double* Aout, double* lams, double* P,
                            double* Q, double tol, int max_iter, int* iters);
int gauge_fix_impl(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, int d, int D,
                   const double* a_ref, const double* a_new, double* U, double tol, int max_iter,
                   double* fidelity, int* iters);
int gauge_fix_1d(tn_ctx* ctx, int method, int chi, int d, const double* a_ref,
                 const double* a_new, double* U, double tol, int max_iter, double* fidelity,
                 int* iters);
int bond_env_truncate_impl(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, int d, int D,
                           int Dk, int De, const double* Theta, int chi, const double* C,
                           const double* T, const double* Psu, const double* Qsu,
                           double* P, double* Q,
                           int max_passes, int max_sweeps, double tol, double* cost, int* passes,
                           int* sweeps);
int bond_environment_impl(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, int d, int D,
                          int Dk, int De, const double* Theta, int chi, const double* C,
                          const double* T, const double* Psu, const double* Qsu,
                          const double* P, const double* Q,
                          int slot, double* N_out, double* M_out);
int fu_gauge_start_impl(tn_ctx* ctx, int nlink, int Dk, int D, int kappa, const double* P,
                        const double* Q, const double* Pc, const double* Qc, double* U0);
int fu_renormalized_gate_impl(tn_ctx* ctx, int nlink, int Dk, int D, const double* P,
                              const double* Q, const double* Pc, const double* Qc, const double* U,
                              double* Rf, double* Lf);
int ipeps_energy_impl(tn_ctx* ctx, int Lx, int Ly, int D, int d, int nsite, const double* sites,
                      const int* cell, int chi, const double* C, const double* T, double J,
                      double h, double* energy);

int energy_grad_impl(tn_ctx* ctx, int D, int d, double J, double h, const double* A, int chi,
                     const double* C0, const double* T0, int n_iter, int ckpt, int prec, double eps,
                     double* energy, double* dEdA);

int ws_reserve(tn_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->arena_size) return TN_OK;
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (ctx->arena) TN_HIP(ctx, hipFree(ctx->arena));
  ctx->arena = nullptr;
  ctx->arena_size = 0;
  const size_t want = bytes + bytes / 8;
  if (hipMalloc(&ctx->arena, want) != hipSuccess) {
    ctx->arena = nullptr;
    (void)hipGetLastError();
    TN_FAIL(ctx, TN_ENOMEM, "cannot allocate %zu bytes of workspace", want);
  }
  ctx->arena_size = want;
  ctx->arena_off = 0;
  return TN_OK;
}

void* ws_alloc_bytes(tn_ctx* ctx, size_t bytes) {
  const size_t off = (ctx->arena_off + 255) & ~size_t(255);
  if (off + bytes > ctx->arena_size) {
    // sticky: every later request fails too, so checking the last pointer
    // of a group of allocations is enough
    ctx->err = "workspace arena exhausted";
    ctx->arena_off = ctx->arena_size;
    return nullptr;
  }
  ctx->arena_off = off + bytes;
  return ctx->arena + off;
}

int keep_buffer(tn_ctx* ctx, const std::string& key, size_t bytes, void** ptr, bool* fresh) {
  auto it = ctx->keep.find(key);
  if (it != ctx->keep.end() && it->second.second == bytes) {
    *ptr = it->second.first;
    if (fresh) *fresh = false;
    return TN_OK;
  }
  if (it != ctx->keep.end()) {
    TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
    TN_HIP(ctx, hipFree(it->second.first));
    ctx->keep.erase(it);
  }
  void* p = nullptr;
  TN_HIP(ctx, hipMalloc(&p, bytes));
  ctx->keep[key] = {p, bytes};
  *ptr = p;
  if (fresh) *fresh = true;
  return TN_OK;
}

extern "C" {

int tn_create(tn_ctx** out, void* hip_stream) {
  if (!out) return TN_EINVAL;
  tn_ctx* ctx = new tn_ctx();
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  // the fixed scratch of the allocation-free calls: its address on this
  // device, taken once per device with the device current
  if (hipGetDevice(&ctx->device) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&ctx->host_scratch),
                    TN_HOST_SCRATCH * sizeof(double)) != hipSuccess ||
      noalloc_scratch_init(ctx->device) != TN_OK) {
    (void)hipGetLastError();
    delete ctx;
    *out = nullptr;
    return TN_EHIP;
  }
  *out = ctx;
  return TN_OK;
}

int tn_destroy(tn_ctx* ctx) {
  if (!ctx) return TN_OK;
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->side) {
    (void)hipStreamSynchronize(ctx->side);
    (void)hipStreamDestroy(ctx->side);
  }
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  if (ctx->arena) (void)hipFree(ctx->arena);
  for (auto& kv : ctx->tables) (void)hipFree(kv.second);
  for (auto& kv : ctx->keep) (void)hipFree(kv.second.first);
  for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->host_scratch) (void)hipHostFree(ctx->host_scratch);
  delete ctx;
  return TN_OK;
}

const char* tn_last_error(const tn_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

const char* tn_version(void) { return "itebd-mi355x 0.1 (gfx950)"; }

int ctmrg_iterate(tn_ctx* ctx, int Lx, int Ly, int D, int d, int nsite, const double* sites,
                  const int* cell, int chi, double* C, double* T, int max_iter, double tol,
                  int precision, int n_polish_fp64, int* iters, double* delta) {
  if (!ctx) return TN_EINVAL;
  ctx->err.clear();
  if (max_iter < 1) TN_FAIL(ctx, TN_EINVAL, "max_iter must be >= 1");
  if (precision != TN_FP64 && precision != TN_FP32 && precision != TN_BF16)
    TN_FAIL(ctx, TN_EINVAL, "unknown precision %d", precision);
  if (n_polish_fp64 < 0) TN_FAIL(ctx, TN_EINVAL, "n_polish_fp64 must be >= 0");
  return ctmrg_run_impl(ctx, Lx, Ly, D, d, nsite, sites, cell, chi, C, T, max_iter, tol, 0, 0,
                        iters, delta, precision, n_polish_fp64);
}

int ctmrg_moves(tn_ctx* ctx, int Lx, int Ly, int D, int d, int nsite, const double* sites,
                const int* cell, int chi, double* C, double* T, int n_moves, int first_dir,
                int precision) {
  if (!ctx) return TN_EINVAL;
  ctx->err.clear();
  if (n_moves < 1) TN_FAIL(ctx, TN_EINVAL, "n_moves must be >= 1");
  if (first_dir < 0 || first_dir > 3) TN_FAIL(ctx, TN_EINVAL, "first_dir must be 0..3");
  if (precision != TN_FP64 && precision != TN_FP32 && precision != TN_BF16)
    TN_FAIL(ctx, TN_EINVAL, "unknown precision %d", precision);
  return ctmrg_run_impl(ctx, Lx, Ly, D, d, nsite, sites, cell, chi, C, T, 0, 0.0, n_moves,
                        first_dir, nullptr, nullptr, precision, 0);
}

int ipeps_rdms(tn_ctx* ctx, int Lx, int Ly, int D, int d, int nsite, const double* sites,
               const int* cell, int chi, const double* C, const double* T, double* rho1,
               double* rhoh, double* rhov) {
  if (!ctx) return TN_EINVAL;
  ctx->err.clear();
  return ipeps_rdms_impl(ctx, Lx, Ly, D, d, nsite, sites, cell, chi, C, T, rho1, rhoh, rhov);
}

int tn_gemm(tn_ctx* ctx, int M, int N, int K, const double* A, int lda, int ta, const double* B,
            int ldb, int tb, double* C, int ldc, double alpha, double beta, int precision) {
  if (!ctx) return TN_EINVAL;
  ctx->err.clear();
  if (M < 0 || N < 0 || K < 0 || !A || !B || !C) TN_FAIL(ctx, TN_EINVAL, "bad gemm arguments");
  if (precision != TN_FP64 && precision != TN_FP32 && precision != TN_BF16)
    TN_FAIL(ctx, TN_EINVAL, "unknown precision %d", precision);
  TN_TRY(gemm(ctx, M, N, K, A, lda, ta != 0, B, ldb, tb != 0, C, ldc, alpha, beta, 1, 0, 0, 0,
              precision));
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return TN_OK;
}

size_t tn_env1d_size(int chi, int d) { return env1d_doubles(chi, d); }

int tm_fixed_point(tn_ctx* ctx, int n_sites, int chi, int d, const double* ket, const double* bra,
                   double* vl, double* vr, double* eta, double tol, int max_iter, int* iters,
                   int flags) {
  if (!ctx) return TN_EINVAL;
  ctx->err.clear();
  return tm_fixed_point_impl(ctx, n_sites, chi, d, ket, bra, vl, vr, eta, tol, max_iter, iters,
                             flags);
}

int tm_fixed_point_noalloc(tn_ctx* ctx, int n_sites, int chi, int d, const double* ket,
                           const double* bra, double* vl, double* vr, double* eta, double tol,
                           int max_iter, int* iters, int flags) {
  if (!ctx) return TN_EINVAL;
  ctx->err.clear();
  return tm_fixed_point_noalloc_impl(ctx, n_sites, chi, d, ket, bra, vl, vr, eta, tol, max_iter,
                                     iters, flags);
}

int itebd_step(tn_ctx* ctx, int chi, int d, double* A, double J, double h, double dt, int mode,
               double* env1d, double* lambda_out, double tol, double* trunc_err,
               double* energy_or_null) {
  if (!ctx) return TN_EINVAL;
  ctx->err.clear();
  return itebd_step_impl(ctx, chi, d, A, J, h, dt, mode, env1d, lambda_out, tol, trunc_err,
                         energy_or_null);
}

int ising2d_tm_step(tn_ctx* ctx, int chi, double* A, double beta, int mode, double* env1d,
                    double* lambda_out, double tol, double* trunc_err, double* lnz_or_null) {
  if (!ctx) return TN_EINVAL;
  ctx->err.clear();
  return ising2d_tm_step_impl(ctx, chi, A, beta, mode, env1d, lambda_out, tol, trunc_err,
                              lnz_or_null);
}

int ipeps_cell_links(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, int* nlink,
                     int* links) {
  if (!ctx) {  // host-only: usable without a context (errors give the code only)
    tn_ctx tmp;
    return cell_links_impl(&tmp, Lx, Ly, nsite, cell, nlink, links);
  }
  ctx->err.clear();
  return cell_links_impl(ctx, Lx, Ly, nsite, cell, nlink, links);
}

int bond_environment(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, int d, int D,
                     int Dk, int De, const double* Theta, int chi, const double* C,
                     const double* T, const double* Psu, const double* Qsu,
                     const double* P, const double* Q,
                     int slot, double* N, double* M) {
  if (!ctx) return TN_EINVAL;
  ctx->err.clear();
  return bond_environment_impl(ctx, Lx, Ly, nsite, cell, d, D, Dk, De, Theta, chi, C, T, Psu,
                               Qsu, P, Q, slot, N, M);
}

int fu_gauge_start(tn_ctx* ctx, int nlink, int Dk, int D, int kappa, const double* P,
                   const double* Q, const double* Pc, const double* Qc, double* U0) {
  if (!ctx) return TN_EINVAL;
  ctx->err.clear();
  return fu_gauge_start_impl(ctx, nlink, Dk, D, kappa, P, Q, Pc, Qc, U0);
}

int ipeps_gate(tn_ctx* ctx, int nsite, int D, int d, double J, double h, double dt,
               const double* A, double* Theta) {
  if (!ctx) return TN_EINVAL;
  ctx->err.clear();
  return ipeps_gate_impl(ctx, nsite, D, d, J, h, dt, A, Theta);
}

int ipeps_truncate(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, int d, int D_in,
                   int D_out, const double* Theta, const double* P, const double* Q,
                   double* A_out) {
  if (!ctx) return TN_EINVAL;
  ctx->err.clear();
  return ipeps_truncate_impl(ctx, Lx, Ly, nsite, cell, d, D_in, D_out, Theta, P, Q, A_out);
}

int ipeps_canonicalize(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, int d, int D,
                       int D_keep, const double* A, double* A_out, double* lambdas, double* P,
                       double* Q, double tol, int max_iter, int* iters) {
  if (!ctx) return TN_EINVAL;
  ctx->err.clear();
  return ipeps_canonicalize_impl(ctx, Lx, Ly, nsite, cell, d, D, D_keep, A, A_out, lambdas, P, Q,
                                 tol, max_iter, iters);
}

int gauge_fix(tn_ctx* ctx, int kind, int Lx, int Ly, int nsite, const int* cell, int d, int D,
              const double* a_ref, const double* a_new, double* U, double tol, int max_iter,
              double* fidelity, int* iters) {
  if (!ctx) return TN_EINVAL;
  ctx->err.clear();
  if (kind == TN_GAUGE_2D)
    return gauge_fix_impl(ctx, Lx, Ly, nsite, cell, d, D, a_ref, a_new, U, tol, max_iter,
                          fidelity, iters);
  if (kind == TN_GAUGE_1D || kind == TN_GAUGE_1D_DIRECT)
    return gauge_fix_1d(ctx, kind == TN_GAUGE_1D ? 0 : 1, D, d, a_ref, a_new, U, tol, max_iter,
                        fidelity, iters);
  TN_FAIL(ctx, TN_EINVAL, "unknown gauge_fix kind %d", kind);
}

int bond_env_truncate(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, int d, int D,
                      int Dk, int De, const double* Theta, int chi, const double* C,
                      const double* T, const double* Psu, const double* Qsu,
                      double* P, double* Q, int max_passes,
                      int max_sweeps, double tol, double* cost, int* passes, int* sweeps) {
  if (!ctx) return TN_EINVAL;
  ctx->err.clear();
  return bond_env_truncate_impl(ctx, Lx, Ly, nsite, cell, d, D, Dk, De, Theta, chi, C, T, Psu,
                                Qsu, P, Q, max_passes, max_sweeps, tol, cost, passes, sweeps);
}

int fu_renormalized_gate(tn_ctx* ctx, int nlink, int Dk, int D, const double* P, const double* Q,
                         const double* Pc, const double* Qc, const double* U, double* Rf,
                         double* Lf) {
  if (!ctx) return TN_EINVAL;
  ctx->err.clear();
  return fu_renormalized_gate_impl(ctx, nlink, Dk, D, P, Q, Pc, Qc, U, Rf, Lf);
}

int ipeps_energy(tn_ctx* ctx, int Lx, int Ly, int D, int d, int nsite, const double* sites,
                 const int* cell, int chi, const double* C, const double* T, double J, double h,
                 double* energy) {
  if (!ctx) return TN_EINVAL;
  ctx->err.clear();
  return ipeps_energy_impl(ctx, Lx, Ly, D, d, nsite, sites, cell, chi, C, T, J, h, energy);
}

int energy_grad(tn_ctx* ctx, int D, int d, double J, double h, const double* A, int chi,
                const double* C0, const double* T0, int n_iter, int ckpt_every, int precision,
                double svd_broadening, double* energy, double* dEdA) {
  if (!ctx) return TN_EINVAL;
  ctx->err.clear();
  // the split-K partials and the Jacobi work matrix of the n x n products
  const size_t n = (size_t)chi * D * D;
  TN_TRY(ws_reserve(ctx, 24 * n * n * sizeof(double) + ((size_t)16 << 20)));
  ws_reset(ctx);
  return energy_grad_impl(ctx, D, d, J, h, A, chi, C0, T0, n_iter, ckpt_every, precision,
                          svd_broadening, energy, dEdA);
}

int tn_svd(tn_ctx* ctx, int batch, int m, int n, const double* A, double* U, double* S,
           double* V) {
  if (!ctx) return TN_EINVAL;
  ctx->err.clear();
  if (batch < 1 || m < 1 || n < 1 || m < n || n > 512 || !A || !S)
    TN_FAIL(ctx, TN_EINVAL, "tn_svd needs batch >= 1, m >= n >= 1, n <= 512 (m=%d n=%d)", m, n);
  TN_TRY(ws_reserve(ctx, (size_t)batch * (m * n + n * n) * sizeof(double) + (1 << 20)));
  ws_reset(ctx);
  if (batch == 1 && n > 128)  // one large matrix: spread over the GPU
    TN_TRY(jacobi_svd_large(ctx, m, n, A, n, U, n, S, V, n));
  else
    TN_TRY(jacobi_svd(ctx, batch, m, n, const_cast<double*>(A), n, (long long)m * n, U, n,
                      (long long)m * n, S, n, V, n, (long long)n * n));
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return TN_OK;
}

int tn_cholesky_inv(tn_ctx* ctx, int batch, int k, const double* G, double shift_rel, double* R,
                    double* Rinv, int* info) {
  if (!ctx) return TN_EINVAL;
  ctx->err.clear();
  if (batch < 1 || k < 1 || k > 512 || !G || !R || !Rinv || !info)
    TN_FAIL(ctx, TN_EINVAL, "tn_cholesky_inv needs batch >= 1, 1 <= k <= 512 (k=%d)", k);
  TN_TRY(ws_reserve(ctx, (size_t)batch * sizeof(int) + (1 << 16)));
  ws_reset(ctx);
  int* dinfo = ws_alloc<int>(ctx, batch);
  if (!dinfo) TN_FAIL(ctx, TN_ENOMEM, "workspace exhausted");
  TN_TRY(cholesky_inv(ctx, k, G, shift_rel, R, Rinv, dinfo, batch));
  TN_HIP(ctx, hipMemcpyAsync(info, dinfo, batch * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return TN_OK;
}

int tn_clear_cache(tn_ctx* ctx) {
  if (!ctx) return TN_EINVAL;
  ctx->err.clear();
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (auto& kv : ctx->keep) TN_HIP(ctx, hipFree(kv.second.first));
  ctx->keep.clear();
  ctx->keep_flags.clear();
  return TN_OK;
}

int tn_prof_enable(tn_ctx* ctx, int on) {
  if (!ctx) return TN_EINVAL;
  unsigned long long sw = 0;
  TN_TRY(jacobi_sweeps_read(ctx, &sw));  // restart the sweep counter too
  ctx->prof = on != 0;
  ctx->ev_used = 0;
  ctx->prof_flops.clear();
  ctx->prof_bytes = 0.0;
  ctx->svd_iters = ctx->svd_calls = ctx->svd_unconverged = ctx->svd_explicit = ctx->moves = 0;
  return TN_OK;
}

int tn_prof_read(tn_ctx* ctx, double* gemm_ms, double* gemm_flops, long long* gemm_launches,
                 long long* counters) {
  if (!ctx) return TN_EINVAL;
  ctx->err.clear();
  TN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  double ms = 0.0, fl = 0.0;
  for (size_t i = 0; i + 1 < ctx->ev_used; i += 2) {
    float t = 0.f;
    TN_HIP(ctx, hipEventElapsedTime(&t, ctx->ev_pool[i], ctx->ev_pool[i + 1]));
    ms += t;
  }
  for (double f : ctx->prof_flops) fl += f;
  if (gemm_ms) *gemm_ms = ms;
  if (gemm_flops) *gemm_flops = fl;
  if (gemm_launches) *gemm_launches = (long long)ctx->prof_flops.size();
  unsigned long long sw = 0;
  TN_TRY(jacobi_sweeps_read(ctx, &sw));
  if (counters) {
    counters[5] = (long long)sw;
    counters[0] = ctx->moves;
    counters[1] = ctx->svd_calls;
    counters[2] = ctx->svd_iters;
    counters[3] = ctx->svd_unconverged;
    counters[4] = ctx->svd_explicit;
    counters[6] = (long long)ctx->prof_bytes;
  }
  ctx->ev_used = 0;
  ctx->prof_flops.clear();
  ctx->prof_bytes = 0.0;
  ctx->svd_iters = ctx->svd_calls = ctx->svd_unconverged = ctx->svd_explicit = ctx->moves = 0;
  return TN_OK;
}

}  // extern "C"
