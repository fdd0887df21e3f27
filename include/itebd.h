/*
 * C ABI of the MI355X environment-recycled imaginary-time TEBD library.
 *
 * Method: Phien, McCulloch and Vidal, "Faster convergence of imaginary time
 * evolution tensor network algorithms by recycling the environment"
 * (arXiv:1411.0391).
 *
 * Conventions shared by every call
 * --------------------------------
 * - All tensors are float64, C-contiguous (row-major), real.
 * - Tensor arguments are DEVICE pointers owned by the caller (e.g. a torch
 *   tensor's data_ptr()); the library never frees or keeps them past the
 *   call.  Small descriptors (unit cells) and scalar outputs are HOST
 *   pointers, as marked.
 * - Every call is ordered on the context's HIP stream and returns after its
 *   host scalar outputs are valid (the call synchronises that stream).
 * - Return codes: TN_OK (0); TN_NOT_CONVERGED (1): outputs hold the last
 *   iterate, the tolerance was not met; negative codes: outputs unspecified,
 *   tn_last_error() has the message.
 * - One context per host thread; calls on one context must not overlap.
 * - iPEPS site tensors A[s][l][r][d][u] (physical, left, right, down, up).
 * - Unit cell: Lx x Ly positions, position p = y*Lx + x (x right, y down,
 *   periodic); cell[p] is the index of the site tensor at p.
 * - CTM environment per position: corners C[p][k][chi][chi] and edges
 *   T[p][k][chi][D][D][chi], k = 0..3 for C1..C4 (top-left, top-right,
 *   bottom-right, bottom-left) and T1..T4 (top, right, bottom, left); the
 *   two boundary legs of each tensor are ordered clockwise around the ring
 *   C1 T1 C2 T2 C3 T3 C4 T4, an edge's middle legs are (ket, bra).
 */
#ifndef ITEBD_H
#define ITEBD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tn_ctx tn_ctx;

enum {
  TN_OK = 0,
  TN_NOT_CONVERGED = 1,
  TN_EINVAL = -1,
  TN_EHIP = -2,
  TN_ENUMERIC = -3,
  TN_ENOMEM = -4
};

/* Bulk-contraction precision of ctmrg_iterate (factorisations stay FP64). */
enum { TN_FP64 = 0, TN_FP32 = 1, TN_BF16 = 2 };

/* Create a context on the current HIP device.  hip_stream may be NULL (the
 * null stream) or a hipStream_t owned by the caller.  The context may also
 * create one stream of its own (default priority, on first use) for work
 * that overlaps the caller's stream inside a call; every such fork is
 * joined back to hip_stream by an event before the work that depends on
 * it, and tn_destroy releases it.  Errors: TN_EHIP. */
int tn_create(tn_ctx** ctx, void* hip_stream);

/* Release the context and everything it allocated. */
int tn_destroy(tn_ctx* ctx);

/* Message of the last failed call on this context ("" if none).  The
 * string stays valid until the next call on the context. */
const char* tn_last_error(const tn_ctx* ctx);

/* Library version string. */
const char* tn_version(void);

/*
 * ctmrg_iterate -- corner transfer matrix environment of an iPEPS (Sec. VI B,
 * Fig. 21(a) of the paper).
 *
 * Directional CTMRG on an Lx x Ly cell: one iteration is a left, up, right
 * and down move, each absorbing every column (row) of the cell in turn; a
 * move computes, for each row cut, the projector pair from the truncated SVD
 * of the product of the two halves of the 2x2 block of enlarged corners,
 * P = R_d V S^-1/2 and Pt = S^-1/2 W^T R_u^T with R_u^T R_d = W S V^T, and
 * renormalises C1, T4, C4 of the next column.  New tensors are scaled to
 * unit Frobenius norm.  Convergence: delta = max over corners of the l2
 * change of the corner's singular values normalised to unit l2 norm, per
 * iteration; stops when delta < tol or after max_iter iterations.
 *
 *   Lx, Ly        cell size (>= 1)
 *   D, d          PEPS bond and physical dimension
 *   nsite         number of distinct site tensors
 *   sites         device [nsite][d][D][D][D][D]
 *   cell          host  [Lx*Ly] site index per position, each < nsite
 *   chi           environment bond dimension (chi <= chi*D*D)
 *   C, T          device in/out, shapes above; the input is the start
 *   max_iter      maximum iterations (>= 1)
 *   tol           convergence tolerance on delta
 *   precision     TN_FP64, TN_FP32 or TN_BF16 for the bulk contractions
 *                 (enlarged corners, renormalisation); SVDs stay FP64
 *   n_polish_fp64 with a reduced precision, the minimum number of final
 *                 FP64 iterations.  The reduced-precision phase stops at
 *                 delta < sw (1e-6 FP32, 1e-3 BF16), or when delta stops
 *                 improving at the precision's noise floor (after five
 *                 iterations, the best delta of the last three is not below
 *                 0.7 times the best before them), or after max_iter
 *                 iterations; its projector SVDs stop at residuals of 2e-5
 *                 (FP32) or 2e-2 (BF16) times s_1, or after 12 (6) subspace
 *                 iterations.  The FP64 phase then runs at least
 *                 n_polish_fp64 iterations and until delta < tol (at most
 *                 max_iter + n_polish_fp64 iterations in all).  iters counts
 *                 both phases.  The FP64 iterations also stop (TN_NOT_CONVERGED)
 *                 when delta stalls: after 20 of them, the best delta of the
 *                 last 10 is not below 0.9 times the best before them
 *   iters, delta  host out: iterations done and the last delta
 * Returns TN_OK, TN_NOT_CONVERGED, TN_EINVAL (bad sizes or pointers),
 * TN_ENUMERIC (non-finite values or a failed factorisation), TN_EHIP.
 */
int ctmrg_iterate(tn_ctx* ctx, int Lx, int Ly, int D, int d, int nsite, const double* sites,
                  const int* cell, int chi, double* C, double* T, int max_iter, double tol,
                  int precision, int n_polish_fp64, int* iters, double* delta);

/*
 * ctmrg_moves -- run exactly n_moves directional moves (no convergence test),
 * starting with direction first_dir (0 left, 1 up, 2 right, 3 down) and
 * column 0, in the order ctmrg_iterate uses.  For measurement and parity
 * checks of single moves.  Arguments as ctmrg_iterate.
 */
int ctmrg_moves(tn_ctx* ctx, int Lx, int Ly, int D, int d, int nsite, const double* sites,
                const int* cell, int chi, double* C, double* T, int n_moves, int first_dir,
                int precision);

/*
 * ipeps_rdms -- reduced density matrices from a CTM environment (used for
 * the TFIM energy and magnetisation, Sec. VI D).
 *   rho1 device out [Lx*Ly][d][d]          one-site, at each position
 *   rhoh device out [Lx*Ly][d*d][d*d]      position with its right neighbour
 *   rhov device out [Lx*Ly][d*d][d*d]      position (top) with the one below
 * Each matrix has trace 1; two-site matrices are indexed (s1 s2),(s1' s2').
 */
int ipeps_rdms(tn_ctx* ctx, int Lx, int Ly, int D, int d, int nsite, const double* sites,
               const int* cell, int chi, const double* C, const double* T, double* rho1,
               double* rhoh, double* rhov);

/*
 * tm_fixed_point -- the 1D environment: dominant left and right eigenvectors
 * of the unit-cell transfer matrix of an iMPS (Sec. III A; with different ket
 * and bra tensors the mixed transfer matrix of Eq. (iMPSDM1)).
 *   n_sites, chi, d  cell length, bond and physical dimension
 *   ket, bra         device [n_sites][chi][d][chi] (lambda absorbed, A form)
 *   vl, vr           device out [chi][chi], indexed (ket, bra):
 *                    eta vl = sum_s K^T vl B over the cell,
 *                    eta vr = sum_s K vr B^T over the cell (last site first);
 *                    |vl|_F = 1, Tr(vl) > 0, sum(vl * vr) = 1
 *   eta              host out: dominant eigenvalue
 *   tol, max_iter    power-iteration stop: iterate moves by < tol (2-norm)
 *   iters            host out: iterations used
 *   flags            bit 0: start from the vl, vr passed in
 * Returns TN_OK, TN_NOT_CONVERGED (e.g. a complex dominant pair of the mixed
 * transfer matrix), TN_EINVAL, TN_ENUMERIC, TN_EHIP.
 */
int tm_fixed_point(tn_ctx* ctx, int n_sites, int chi, int d, const double* ket, const double* bra,
                   double* vl, double* vr, double* eta, double tol, int max_iter, int* iters,
                   int flags);

/*
 * tm_fixed_point_noalloc -- tm_fixed_point for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation): the same arguments, kernels and results, with
 * the iterate pair, the eigenvalue and iteration outputs and the kernels'
 * working set in a fixed device array of 4 MiB (2^19 doubles) that the
 * library holds on each GPU until the process ends; the call itself
 * allocates nothing.  It needs 2 chi^2 + 32 doubles, plus 2 (2 n_sites d
 * + d + 2) chi^2 when that working set exceeds 150 KiB of LDS (the
 * two-site, d = 2 cell: chi <= 40 in LDS, chi <= 142 in all); larger
 * problems return TN_EINVAL.  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (several contexts or streams) race and give undefined
 * results.  The array keeps the last call's contents; nothing in it needs
 * clearing, the kernels write what they read.
 */
int tm_fixed_point_noalloc(tn_ctx* ctx, int n_sites, int chi, int d, const double* ket,
                           const double* bra, double* vl, double* vr, double* eta, double tol,
                           int max_iter, int* iters, int flags);

/* Size in doubles of the env1d workspace of itebd_step for bond chi. */
size_t tn_env1d_size(int chi, int d);

/* itebd_step modes */
enum {
  TN_PLAIN = 0,
  TN_RECYCLE_BUILD = 1,
  TN_RECYCLE_APPLY = 2,
  TN_RECYCLE_LIMIT = 3,
  TN_RECYCLE_BUILD_DIRECT = 4
};

/*
 * itebd_step -- one imaginary-time step of the transverse-field Ising chain
 * H = -J sum sz sz - h sum sx on a two-site iMPS (Sec. V).  The state is in
 * the symmetric A form (sqrt(lambda) Gamma sqrt(lambda)).
 *   A          device in/out [2][chi][d][chi] (d = 2); site 0 then site 1
 *   dt         time step; the iMPO of Eq. (iMPO1) (second-order Trotter)
 *   mode       TN_PLAIN: Theta = g A, environment = transfer-matrix fixed
 *              points of the Theta chain, truncation A = Q Theta P
 *              (Eq. (EqCanoPQ1)) on both bonds.
 *              TN_RECYCLE_BUILD: an environment step of the recycling scheme
 *              (Sec. V B (i)-(iii)): A_0 is brought to canonical form, the
 *              plain truncation of g A_0 is brought to canonical form
 *              (Qc, Pc; sign rule on the columns of Pc), its gauge is fixed
 *              against A_0 by the alternating Procrustes maximisation of the
 *              fidelity (start: kappa = 0 blocks of P Pc and Qc Q), and the
 *              renormalized gate G = U^T (Qc Q) g (P Pc) U is stored in
 *              env1d; the new state is G A_0.  Needs chi <= 64.
 *              TN_RECYCLE_BUILD_DIRECT: the same environment step with the
 *              gauge fixed by the direct method (Sec. III B 1, Eq.
 *              (iMPSDM1)): per bond U is the orthogonal polar factor of the
 *              transposed dominant left eigenvector of the mixed transfer
 *              matrix of (A_0, canonical truncated state), the pair's sign
 *              taken with a positive fidelity.  Stays at the fixed point
 *              where the Procrustes iteration stalls (a Schmidt spectrum
 *              with near-degenerate pairs, a gate far from the identity).
 *              TN_RECYCLE_APPLY: A <- G A with the stored G (no environment);
 *              TN_EINVAL if no build step has stored one; lambda_out is not
 *              written and trunc_err is 0.
 *              TN_RECYCLE_LIMIT: the limit N_Re -> infinity of applying the
 *              stored G (Sec. V C): each site becomes the dominant
 *              eigenvector of its map A_X -> G A_X, unit norm, sign with a
 *              positive overlap with the site passed in; computed by
 *              squaring the dense map with normalisation until G v = rho v
 *              to 1e-10 (relative); TN_NOT_CONVERGED when G has no simple
 *              real dominant eigenvalue (outputs then hold the last
 *              iterate); otherwise as TN_RECYCLE_APPLY
 *   env1d      device workspace of tn_env1d_size(chi, d) doubles, owned by
 *              the caller, zero-filled before the first step; carries warm
 *              starts between steps
 *   lambda_out device out [2][chi] (may be NULL): kept spectra of bonds 0
 *              (after site 0) and 1, unit l2 norm (after a build step: the
 *              canonical spectra of the truncated state)
 *   tol        fixed-point tolerance (the bond environments come from
 *              restarted Arnoldi: Arnoldi residual below tol times the
 *              Ritz value, or below 100 tol while no longer halving per
 *              restart)
 *   trunc_err  host out: discarded weight summed over the two bonds
 *   energy_or_null host out (may be NULL): energy per site of the new state
 * Returns TN_OK, TN_NOT_CONVERGED (a fixed point hit its iteration cap),
 * TN_EINVAL, TN_ENUMERIC, TN_EHIP.
 */
int itebd_step(tn_ctx* ctx, int chi, int d, double* A, double J, double h, double dt, int mode,
               double* env1d, double* lambda_out, double tol, double* trunc_err,
               double* energy_or_null);

/*
 * ising2d_tm_step -- one step of the power method for the partition function
 * of the classical square-lattice Ising model (J = 1, inverse temperature
 * beta): the two-site iMPS A encodes the dominant eigenvector of the
 * row-to-row transfer matrix, which takes the place of the imaginary-time
 * operator (Sec. I), and the environment can be recycled as in Sec. V.
 * The transfer matrix with the vertical bonds between two rows and half of
 * each row's horizontal bonds is c^L G, c = sqrt(2 sinh 2 beta), G the
 * second-order gate of the transverse-field chain at dt J = beta,
 * dt h = K* (tanh K* = exp(-2 beta)); so this is itebd_step with that gate.
 *   chi, A, mode, env1d, lambda_out, tol, trunc_err  as for itebd_step
 *              (d = 2; every mode, TN_RECYCLE_LIMIT included)
 *   beta       inverse temperature, > 0
 *   lnz_or_null host out (may be NULL): ln Z per site of the model (minus
 *              beta times the free energy per site) from the new state:
 *              ln c + ln mu, mu the per-site Rayleigh quotient of G, i.e.
 *              the square root of the ratio of the dominant eigenvalues of
 *              the two-site transfer matrices of (G A, A) and (A, A)
 * Returns as itebd_step; TN_EINVAL for beta <= 0.
 */
int ising2d_tm_step(tn_ctx* ctx, int chi, double* A, double beta, int mode, double* env1d,
                    double* lambda_out, double tol, double* trunc_err, double* lnz_or_null);

/*
 * ---------------------------------------------------------------------------
 * Full update of an iPEPS (Sec. VI B, VI C), canonical form (Sec. IV A) and
 * gauge fixing (Sec. IV B).
 *
 * Links of a unit cell: enumerated in first-seen order over the positions
 * p = 0, 1, ..., the right link of a position before its down link; link b
 * joins leg l1 (r or d) of site s1 with leg l2 (l or u) of site s2 (legs
 * numbered 1 l, 2 r, 3 d, 4 u as tensor axes).  Per-link matrices: the first
 * end carries P[b] (n_old x n_new, applied as new = P^T old on that leg), the
 * second end Q[b] (n_new x n_old, new = Q old): A~ = Q Theta P.
 * ---------------------------------------------------------------------------
 */

/* ipeps_cell_links -- the link enumeration above, for the caller's
 * bookkeeping.  nlink host out; links host out [64][4] = (s1, l1, s2, l2).
 * Host-only: ctx may be NULL.  Errors: TN_EINVAL for a cell that puts two
 * links on one leg or leaves a site out. */
int ipeps_cell_links(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, int* nlink,
                     int* links);

/*
 * ipeps_gate -- Theta = g A (Sec. VI A, Fig. 20): the TFIM iPEPO of one
 * second-order Trotter step (half field steps exp(dt h sx / 2) on both sides
 * of the four bond factors of exp(dt J sz sz), split by operator SVD into
 * kappa = 2 terms) applied to every site tensor.
 *   A      device [nsite][d][D][D][D][D], d = 2
 *   Theta  device out [nsite][d][2D][2D][2D][2D]; each bond index is
 *          (D index, kappa index) with the kappa index fastest
 */
int ipeps_gate(tn_ctx* ctx, int nsite, int D, int d, double J, double h, double dt,
               const double* A, double* Theta);

/*
 * ipeps_truncate -- A~ = Q Theta P on every link (Sec. VI B), each site then
 * scaled to unit Frobenius norm.  Also applies the renormalized gate's
 * factors (Sec. VI C) when called with Rf, Lf as P, Q.
 *   Theta  device [nsite][d][D_in]^4;  P device [nlink][D_in][D_out];
 *   Q      device [nlink][D_out][D_in]; A_out device out [nsite][d][D_out]^4
 */
int ipeps_truncate(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, int d, int D_in,
                   int D_out, const double* Theta, const double* P, const double* Q,
                   double* A_out);

/*
 * ipeps_canonicalize -- canonical form of an iPEPS (Sec. IV A, Eqs. (17)-(20))
 * by the paper's iteration on every link at once: per link the Gram matrices
 * V1, V2 of the two ends (lambda on the other three legs) give V1 = Y^T Y,
 * V2 = X X^T, the SVD Y lambda X = U S V^T gives the transforms Y^+ U and
 * V^T X^+ and the new spectrum S / |S|; starting from flat spectra, until
 * the spectra move by less than tol (max norm).  Pseudo-inverse square roots
 * drop eigenvalues below 1e-14 of the largest; the columns of each transform
 * Y^+ U are sign-fixed (first entry within 1e-8 of the largest magnitude
 * positive).
 *   A        device [nsite][d][D]^4, the state in A form
 *   A_out    device out (may be NULL; needs D_keep = D): the canonical A form
 *            A1 = Qc A Pc, unit norm per site
 *   lambdas  device out (may be NULL) [nlink][D]: spectra, unit l2 norm
 *   P, Q     device out [nlink][D][D_keep], [nlink][D_keep][D]: the first
 *            D_keep columns of Pc = TR sqrt(lambda) and rows of
 *            Qc = sqrt(lambda) TL, TR and TL the accumulated transforms of
 *            the two ends.  With D_keep < D this is the simple-update style
 *            pre-truncation of a gated state Theta (keep the D_keep largest
 *            Schmidt values of every link)
 *   tol, max_iter, iters (host out)
 * Returns TN_OK or TN_NOT_CONVERGED (outputs from the last iterate).
 */
int ipeps_canonicalize(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, int d, int D,
                       int D_keep, const double* A, double* A_out, double* lambdas, double* P,
                       double* Q, double tol, int max_iter, int* iters);

/* gauge_fix kinds */
enum { TN_GAUGE_2D = 0, TN_GAUGE_1D = 1, TN_GAUGE_1D_DIRECT = 2 };

/*
 * gauge_fix -- fix the gauge freedom between two tensor networks that
 * represent one state (Sec. III B for an iMPS, Sec. IV B for an iPEPS),
 * with one orthogonal U_b per link (real arithmetic: unitary means
 * orthogonal), U_b applied as new = U_b old on both legs of link b.
 *   kind = TN_GAUGE_2D: an iPEPS cell (Lx, Ly, nsite, cell as for the
 *          full-update calls, bond D, a_ref, a_new [nsite][d][D]^4, nsite
 *          <= 30).  Maximises the fidelity of Eq. (25),
 *          F = sum_s <a_new_s | U(a_ref_s)> / sum_s |a_ref_s| |a_new_s|, by
 *          alternating Procrustes steps (Sec. IV B): each link in turn, the
 *          other factors fixed, U_b = W V^T from the SVD of the linear
 *          coefficient W S V^T; from the U passed in until F changes by less
 *          than tol in a pass over the links.
 *   kind = TN_GAUGE_1D: the two-site iMPS cell (Lx, Ly, nsite, cell ignored;
 *          D = chi; a_ref, a_new [2][chi][d][chi] in A form, site 0 with
 *          bond 1 on its left and bond 0 on its right, so a_new_X ~
 *          U[left] a_ref_X U[right]^T).  The iterative method (Sec. III B 2,
 *          Eq. (15)) as for 2D, from the U passed in.
 *   kind = TN_GAUGE_1D_DIRECT: the same cell by the direct method (Sec.
 *          III B 1, Eq. (iMPSDM1)): per bond the dominant left eigenvector
 *          X of the mixed transfer matrix (ket a_ref, bra a_new) equals
 *          w U^T with w the positive fixed point of a_ref, so U is the
 *          orthogonal polar factor of X^T; the sign of the pair is taken
 *          with F > 0.  U is output only.  The eigenvectors of both
 *          bonds come from one restarted-Arnoldi launch: it stops when
 *          the Arnoldi residual is below tol times the Ritz value, or
 *          below 100 tol times it while no longer halving per restart
 *          (its rounding floor) (tol <= 0: 1e-14); max_iter bounds the
 *          transfer-matrix applications.  chi <= 64 for both 1D kinds.
 *   U             device in/out [nlink][D][D] (1D: [2][chi][chi])
 *   fidelity, iters  host out
 * Returns TN_OK, TN_NOT_CONVERGED, TN_EINVAL, TN_ENUMERIC, TN_EHIP.
 */
int gauge_fix(tn_ctx* ctx, int kind, int Lx, int Ly, int nsite, const int* cell, int d, int D,
              const double* a_ref, const double* a_new, double* U, double tol, int max_iter,
              double* fidelity, int* iters);

/*
 * The full-update truncation works on a 2x2 block of sites (Sec. VI B,
 * Fig. 21(a)): positions TL = (0, 0), TR = (1, 0), BR = (1, 1), BL = (0, 1)
 * of the cell, surrounded by their CTM corners and edges.  Its four internal
 * links are the slots, visited in the order
 *   0 top    (TL.r - TR.l),   1 left  (TL.d - BL.u),
 *   2 bottom (BL.r - BR.l),   3 right (TR.d - BR.u),
 * the first end of each carrying P.  The block's legs that face the
 * environment carry the pre-truncation (Psu, Qsu) the environment was
 * computed for.  A cell is accepted when every one of its links is a slot
 * (the checkerboard: slot k is link k; the 1 x 1 cell: slots 0, 2 are link 0
 * and slots 1, 3 link 1); other cells give TN_EINVAL.
 */

/*
 * bond_env_truncate -- the full-update truncation of every link (Sec. VI B,
 * Eqs. (var), (var1)): minimises the block cost
 *   f(zeta) = <Psi_g|Psi_g> - 2 <Psi_g|Psi_zeta> + <Psi_zeta|Psi_zeta>
 * over zeta = (P, Q) of the four slots, Psi_g having every internal link at
 * the full bond Dk and Psi_zeta each truncated by its (P, Q).  Cycles over
 * the slots; a visit builds the slot's two environments from the current
 * zeta (bond_environment) and makes up to max_sweeps ALS sweeps: P = R^-1 S
 * with Q fixed, then Q with P fixed, each solve on R + 1e-14 tr(R) I by
 * Gaussian elimination with partial pivoting (R is indefinite when the
 * environment is not positive), then the pair balanced through the SVD of
 * P Q; a visit stops early when a sweep changes f by less than
 * tol <Psi_g|Psi_g>, and the cycles stop when one changes f by less than
 * that, or after max_passes.  Each update minimises f exactly in its
 * variable, so f does not increase.  max_sweeps = 1 is the section's order:
 * one P and one Q update per link per cycle.  A link held by two slots (the
 * 1 x 1 cell) gets the mean of their (P, Q).  kappa D^2 <= 140.
 *   Theta        device [nsite][d][Dk]^4, Dk = kappa D
 *   De           bond of the legs facing the environment, 1 <= De <= Dk
 *   C, T         device, the environment (bond De) of the state those legs
 *                carry: the pre-truncated state (De = D, the O(chi^3 D^6)
 *                form the section proposes), or Theta itself (De = Dk, Psu
 *                and Qsu identities: the O(chi^3 D^6 kappa^6) form)
 *   Psu, Qsu     device [nlink][Dk][De], [nlink][De][Dk]: the pre-truncation
 *   P, Q         device in/out [nlink][Dk][D], [nlink][D][Dk]: start, result
 *   cost         host out (may be NULL) [2]: final f and <Psi_g|Psi_g>
 *   passes, sweeps  host out (may be NULL): cycles and total ALS sweeps
 * Returns TN_OK, TN_EINVAL, TN_ENUMERIC (a singular normal matrix,
 * non-finite values, a zero block norm), TN_EHIP.
 */
int bond_env_truncate(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, int d, int D,
                      int Dk, int De, const double* Theta, int chi, const double* C,
                      const double* T, const double* Psu, const double* Qsu, double* P, double* Q,
                      int max_passes, int max_sweeps, double tol, double* cost, int* passes,
                      int* sweeps);

/*
 * bond_environment -- the two environments of one slot of the truncation
 * block (same arguments as bond_env_truncate; P, Q read only, per link):
 *   N device out [Dk][Dk][Dk][Dk], [i][j][i'][j']: the block with the slot
 *     cut, every other internal link truncated by (P, Q) in both layers;
 *     i, j the ket index of the slot's first and second end, i', j' the bra
 *     index; symmetrised in ket <-> bra
 *   M device out, same layout: the ket layer as for N, the bra layer with
 *     every internal link at the full bond (Psi_g)
 * so that f = <Psi_g|Psi_g> - 2 sum (PQ)_ij M[i][j][a][a] + <PQ|N|PQ> for
 * the slot's (P, Q).  Both carry the sign of the raw network (the
 * normalised boundary leaves a common sign free).
 */
int bond_environment(tn_ctx* ctx, int Lx, int Ly, int nsite, const int* cell, int d, int D,
                     int Dk, int De, const double* Theta, int chi, const double* C,
                     const double* T, const double* Psu, const double* Qsu, const double* P,
                     const double* Q, int slot, double* N, double* M);

/*
 * fu_gauge_start -- start of the gauge fix inside the recycling step
 * (Sec. VI C): for a small time step the renormalized gate is close to the
 * identity, so the kappa = 0 block of the composite truncation maps the old
 * bond basis onto the new one.  Per link, with (P Pc) [Dk][D] and (Qc Q)
 * [D][Dk] and the bond index (i, k) (k the kappa index, fastest):
 * K = B1 / |B1|_F + B2 / |B2|_F, B1[j][i] = (P Pc)[(i, 0)][j],
 * B2[j][i] = (Qc Q)[j][(i, 0)], and U0 = W V^T from K = W S V^T.
 *   P [nlink][Dk][D], Q [nlink][D][Dk], Pc, Qc [nlink][D][D] device;
 *   U0 device out [nlink][D][D]; Dk = kappa D
 */
int fu_gauge_start(tn_ctx* ctx, int nlink, int Dk, int D, int kappa, const double* P,
                   const double* Q, const double* Pc, const double* Qc, double* U0);

/*
 * fu_renormalized_gate -- the per-link factors of the renormalized gate of
 * Sec. VI C, G = U^T (Qc Q) g (P Pc) U: Rf[b] = P[b] Pc[b] U[b] on the first
 * end, Lf[b] = U[b]^T Qc[b] Q[b] on the second end; recycled steps are then
 * ipeps_gate followed by ipeps_truncate with (Rf, Lf).
 *   P [nlink][Dk][D], Q [nlink][D][Dk], Pc, Qc, U [nlink][D][D] (device);
 *   Rf device out [nlink][Dk][D], Lf device out [nlink][D][Dk]
 */
int fu_renormalized_gate(tn_ctx* ctx, int nlink, int Dk, int D, const double* P, const double* Q,
                         const double* Pc, const double* Qc, const double* U, double* Rf,
                         double* Lf);

/*
 * ipeps_energy -- TFIM energy per site from a CTM environment (Sec. VI A,
 * VI D): mean over positions of -J <sz sz> on the position's right and down
 * bonds and -h <sx> on the position, from the reduced density matrices of
 * ipeps_rdms.  d must be 2.  energy host out.
 */
int ipeps_energy(tn_ctx* ctx, int Lx, int Ly, int D, int d, int nsite, const double* sites,
                 const int* cell, int chi, const double* C, const double* T, double J, double h,
                 double* energy);

/*
 * energy_grad -- TFIM energy per site E(A) of a single-site iPEPS (1 x 1
 * cell, Sec. VI A, VI D) after exactly n_iter CTMRG iterations (Sec. VI B,
 * no convergence test) from the environment (C0, T0), and its gradient
 * dE/dA by a hand-written reverse pass through the iterations and the
 * energy.  The environment is an input, not a function of A, so no gradient
 * flows into it.  Projectors come from the full SVD of the explicitly formed
 * ring product of the four enlarged corners (n = chi D^2 <= 512); the SVD
 * adjoint uses the broadened inverse gaps g / (g^2 + svd_broadening
 * (s_i^2 + s_j^2)^2), g = s_j^2 - s_i^2 (0 broadens nothing; exactly
 * degenerate pairs then contribute nothing).  The
 * iterations are checkpointed every ckpt_every iterations and recomputed
 * segment by segment in the reverse pass; the projector factorisations
 * (U, S, V of each move) are kept from the forward pass and reused there,
 * the recomputation being bitwise the forward pass.
 *   A      device [d][D][D][D][D] (s, l, r, d, u); d must be 2
 *   C0, T0 device [4][chi][chi], [4][chi][D][D][chi] (the slots of the one
 *          position, as for ctmrg_iterate)
 *   precision  TN_FP64 (the only one accepted: with FP32 bulk contractions
 *          E(A) after a fixed number of iterations from a random boundary is
 *          ill-conditioned -- the rounding of the early iterations decides
 *          which small singular values of the projector problems come close,
 *          and the inverse gaps of the SVD adjoint amplify it -- so that
 *          form's gradient has no bound to state)
 *   energy host out; dEdA device out, shape of A
 * TN_EINVAL for d != 2, n > 512, n_iter < 0, ckpt_every < 1, a precision
 * other than TN_FP64 or a negative broadening.  Device memory: about 2 GB
 * per checkpoint segment at D = 4, chi = 32, plus 4 n_iter (2 n^2 + n)
 * doubles of kept factorisations (336 MB at n = 512, 20 iterations; when
 * they cannot be allocated the segments recompute them), in chunks of at
 * least 256 MiB that the context keeps for later calls (tn_clear_cache
 * releases them).
 */
int energy_grad(tn_ctx* ctx, int D, int d, double J, double h, const double* A, int chi,
                const double* C0, const double* T0, int n_iter, int ckpt_every, int precision,
                double svd_broadening, double* energy, double* dEdA);

/*
 * tn_gemm -- the library's contraction engine on a plain matrix product, for
 * testing and measurement: C = alpha op(A) op(B) + beta C with row-major
 * storage, op(X) = X or X^T (ta, tb nonzero), leading dimensions lda, ldb,
 * ldc.  All matrices device, FP64.  precision: TN_FP64, or TN_FP32 / TN_BF16
 * (operands rounded to that format on the fly, FP32 accumulation on MFMA,
 * FP64 result).
 */
int tn_gemm(tn_ctx* ctx, int M, int N, int K, const double* A, int lda, int ta, const double* B,
            int ldb, int tb, double* C, int ldc, double alpha, double beta, int precision);

/*
 * tn_svd -- the library's small dense FP64 SVD (one-sided Jacobi, one
 * workgroup per matrix; a single matrix with n > 128 is spread over the
 * whole GPU, one launch per round of column pairs), used for the
 * Rayleigh-Ritz step of the projector SVD, the corner spectra, the canonical-form and gauge-fixing
 * factorisations.  A = U diag(S) V^T for `batch` row-major m x n matrices
 * (m >= n, n <= 512) stored back to back; U [batch][m][n], S [batch][n]
 * (descending), V [batch][n][n]; each column of U sign-fixed so that its
 * first entry within 1e-8 of its largest magnitude is positive.  A is not
 * modified.  U and V may be NULL.  Device pointers.
 */
int tn_svd(tn_ctx* ctx, int batch, int m, int n, const double* A, double* U, double* S,
           double* V);

/*
 * tn_cholesky_inv -- the library's small dense FP64 Cholesky (used by the
 * Cholesky-QR orthonormalisation of the projector SVD and the ALS solves),
 * for testing and measurement: for `batch` row-major k x k matrices G stored
 * back to back (k <= 512), the upper factor R of G + shift I with
 * shift = shift_rel tr(G), G + shift I = R^T R, and its inverse Rinv (device
 * outputs of the same shape).  info (host, batch ints): 0, or the index + 1
 * of the first non-positive pivot (then R and Rinv are unspecified).  With
 * shift_rel = 0 and every entry of G - I within 1e-9 of zero (k <= 128),
 * R = I + U and Rinv = I - U with U the strict upper part of G - I plus
 * half its diagonal, exact up to k max|G - I|^2; a NaN in G always takes
 * the elimination and is reported as a failed pivot.
 */
int tn_cholesky_inv(tn_ctx* ctx, int batch, int k, const double* G, double shift_rel, double* R,
                    double* Rinv, int* info);

/*
 * tn_clear_cache -- drop the state the context keeps between calls: the
 * start bases of the projector SVDs of ctmrg_iterate / ctmrg_moves (kept per
 * cell geometry so that a converging CTMRG restarts its subspace iterations
 * from the previous projectors), and the device memory energy_grad keeps for
 * its tapes.  Results never depend on this state beyond
 * the SVD tolerance; clearing it makes a call independent of earlier calls.
 */
int tn_clear_cache(tn_ctx* ctx);

/*
 * Measurement support.  tn_prof_enable(ctx, 1) starts timing every launch of
 * the contraction kernel with HIP events on the context stream (and resets
 * the counters); tn_prof_read returns, since the last enable/read: total
 * kernel milliseconds, total algorithmic flops (2 M N K per product), the
 * launch count, and counters[7] = {CTMRG moves, projector SVDs, subspace
 * iterations, SVDs above the residual tolerance at their stop, SVDs done by
 * the explicit small-n path, Jacobi sweeps of the small dense SVDs,
 * algorithmic bytes of the timed contractions (8 (MK + KN + MN) per
 * product)}.  Reading resets everything.  Host pointers; any may be NULL.
 */
int tn_prof_enable(tn_ctx* ctx, int on);
int tn_prof_read(tn_ctx* ctx, double* gemm_ms, double* gemm_flops, long long* gemm_launches,
                 long long* counters);

#ifdef __cplusplus
}
#endif

#endif /* ITEBD_H */
