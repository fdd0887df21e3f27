// A network of site tensors joined by links, as the canonical form, the
// truncation and the gauge fixing see it: every site tensor has five axes;
// an axis either carries one end of a link (all links share one dimension n)
// or has a fixed extent (the physical index, or a trivial axis).  A link b
// joins axis a1[b] of site s1[b] (its first end, which carries P: new = P^T
// old) to axis a2[b] of site s2[b] (its second end, which carries Q: new =
// Q old).
#pragma once

#include <array>
#include <vector>

#include "common.h"

struct BondNet {
  int nsite = 0, nl = 0;
  std::vector<std::array<int, 5>> link;  // [site][axis] -> link, or -1
  std::vector<std::array<int, 5>> ext;   // [site][axis] -> extent of a non-link axis
  std::vector<int> s1, a1, s2, a2;
  long long size(int s, int n) const {
    long long t = 1;
    for (int k = 0; k < 5; ++k) t *= link[s][k] >= 0 ? n : ext[s][k];
    return t;
  }
  bool first_end(int s, int ax) const {
    const int b = link[s][ax];
    return b >= 0 && s1[b] == s && a1[b] == ax;
  }
};

// Largest bond of the small per-leg kernels (canonical form, gauge fixing,
// ALS cost), whose n x n tiles live in LDS.
constexpr int TN_SMALL_BOND = 64;

// The two-site iMPS cell [chi][d][chi] (left, physical, right): link 0 joins
// the right leg of site 0 to the left leg of site 1, link 1 the right leg of
// site 1 to the left leg of site 0.
BondNet bondnet_chain2(int d);

// Workspace (bytes) the calls below take from the context arena; the caller
// reserves it (they never grow the arena themselves).
size_t bondnet_canon_bytes(const BondNet& net, int n);
size_t bondnet_gauge_bytes(const BondNet& net, int n);

// Canonical form of the network's A form (Sec. III A in 1D, Sec. IV A in 2D),
// iterated on all links at once from flat spectra until they move by less
// than tol.  Outputs (device, any may be null except Pc, Qc): lams [nl][n],
// Pc [nl][n][n] = TR sqrt(lambda) and Qc = sqrt(lambda) TL with the sign rule
// on the columns of Pc, Aout = Qc A Pc with unit norm per site.
int bondnet_canonicalize(tn_ctx* ctx, const BondNet& net, int n, const double* A, double tol,
                         int max_iter, double* lams, double* Pc, double* Qc, double* Aout,
                         int* iters);

// The canonical sign and scale of a gauge pair on each of nl links (as
// bondnet_canonicalize leaves them): P [nl][n][n] acts on the first ends and
// Q, its inverse up to a factor, on the second.  The sign rule goes on the
// columns of P (the rows of Q flip with them); then P Q = I through its
// trace and |P|_F = |Q|_F.  n <= TN_SMALL_BOND.
int canonical_pq(tn_ctx* ctx, int nl, int n, const double* P, const double* Q, double* Pc,
                 double* Qc);

// out_s = (P on first ends, Q on second ends) in_s, unit norm per site;
// P [nl][n_in][n_out], Q [nl][n_out][n_in]; sc: scratch of two input sites.
int bondnet_truncate(tn_ctx* ctx, const BondNet& net, int n_in, int n_out, const double* in,
                     const double* P, const double* Q, double* out, double* sc);

// Alternating Procrustes maximisation of the fidelity of Eq. (25) (Sec. III B,
// IV B): U [nl][n][n] in (start) / out.
int bondnet_gauge_fix(tn_ctx* ctx, const BondNet& net, int n, const double* a_ref,
                      const double* a_new, double* U, double tol, int max_iter, double* fidelity,
                      int* iters);

// Recycling factors (device): U0 from the kappa = 0 blocks of (P Pc), (Qc Q);
// Rf = P Pc U, Lf = U^T Qc Q.  P [nl][Dk][D], Q [nl][D][Dk], Pc, Qc, U [nl][D][D].
int recycle_gauge_start(tn_ctx* ctx, int nl, int Dk, int D, int kappa, const double* P,
                        const double* Q, const double* Pc, const double* Qc, double* U0);
int recycle_factors(tn_ctx* ctx, int nl, int Dk, int D, const double* P, const double* Q,
                    const double* Pc, const double* Qc, const double* U, double* Rf, double* Lf);
