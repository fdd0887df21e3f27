// Contraction networks of the CTM environment (Sec. VI B, Fig. 21(a)) as
// table-driven contractions, shared by the CTMRG moves, the reduced density
// matrices and the adjoint of both.  Layouts: site A[s][l][r][d][u]; corner
// C[a][b]; edge T[a][ket][bra][b]; n = chi D^2.
#pragma once

#include "common.h"

namespace nets {

// Enlarged corner, ket layer:
// X3[a, b, rk, dk, s, lb, ub] = sum_{lk,uk} X2[a, lk, lb, uk, ub, b] A[s, lk, rk, dk, uk]
inline Contraction corner_ket(long long chi, long long D, long long d) {
  const long long D2 = D * D, D4 = D2 * D2;
  Contraction c;
  c.am = grp({{(int)chi, D4 * chi}, {(int)D, D2 * chi}, {(int)D, chi}, {(int)chi, 1}});
  c.ak = grp({{(int)D, D2 * D * chi}, {(int)D, D * chi}});
  c.bk = grp({{(int)D, D2 * D}, {(int)D, 1}});
  c.bn = grp({{(int)d, D4}, {(int)D, D2}, {(int)D, D}});
  c.cm = grp({{(int)chi, chi * d * D4}, {(int)D, D}, {(int)D, 1}, {(int)chi, d * D4}});
  c.cn = grp({{(int)d, D2}, {(int)D, d * D2 * D}, {(int)D, d * D2}});
  return c;
}

// Enlarged corner, bra layer:
// E[(a, dk, db), (b, rk, rb)] = sum_{s,lb,ub} X3[a, b, rk, dk, s, lb, ub] A[s, lb, rb, db, ub]
inline Contraction corner_bra(long long chi, long long D, long long d, long long n) {
  const long long D2 = D * D, D4 = D2 * D2;
  Contraction c;
  c.am = grp({{(int)chi, chi * d * D4}, {(int)chi, d * D4}, {(int)D, d * D2 * D}, {(int)D, d * D2}});
  c.ak = grp({{(int)d, D2}, {(int)D, D}, {(int)D, 1}});
  c.bk = grp({{(int)d, D4}, {(int)D, D2 * D}, {(int)D, 1}});
  c.bn = grp({{(int)D, D2}, {(int)D, D}});
  c.cm = grp({{(int)chi, D2 * n}, {(int)chi, D2}, {(int)D, D}, {(int)D, D * n}});
  c.cn = grp({{(int)D, 1}, {(int)D, n}});
  return c;
}

// T3 C4 of the left move: Z[a3, (b4, k, b)] = sum_g T3[a3, k, b, g] C4[g, b4]
inline Contraction t3_c4(long long chi, long long D, long long n) {
  const long long D2 = D * D;
  Contraction c;
  c.am = grp({{(int)chi, D2 * chi}, {(int)D, D * chi}, {(int)D, chi}});
  c.ak = grp({{(int)chi, 1}});
  c.bk = grp({{(int)chi, chi}});
  c.bn = grp({{(int)chi, 1}});
  c.cm = grp({{(int)chi, n}, {(int)D, D}, {(int)D, 1}});
  c.cn = grp({{(int)chi, D2}});
  return c;
}

// Edge renormalisation, step 1:
// Y1[c, uk, ub, a, lk, lb] = sum_b PtT[(b, uk, ub), c] T4[a, lk, lb, b]
inline Contraction edge_pt(long long chi, long long D, long long n) {
  const long long D2 = D * D;
  Contraction c;
  c.am = grp({{(int)chi, 1}, {(int)D, D * chi}, {(int)D, chi}});
  c.ak = grp({{(int)chi, D2 * chi}});
  c.bk = grp({{(int)chi, 1}});
  c.bn = grp({{(int)chi, D2 * chi}, {(int)D, D * chi}, {(int)D, chi}});
  c.cm = grp({{(int)chi, D2 * n}, {(int)D, D * n}, {(int)D, n}});
  c.cn = grp({{(int)chi, D2}, {(int)D, D}, {(int)D, 1}});
  return c;
}

// Edge renormalisation, ket layer:
// Y2[c, a, rk, dk, s, lb, ub] = sum_{lk,uk} Y1[c, uk, ub, a, lk, lb] A[s, lk, rk, dk, uk]
inline Contraction edge_ket(long long chi, long long D, long long d, long long n) {
  const long long D2 = D * D, dD4 = d * D2 * D2;
  Contraction c;
  c.am = grp({{(int)chi, D2 * n}, {(int)D, n}, {(int)chi, D2}, {(int)D, 1}});
  c.ak = grp({{(int)D, D}, {(int)D, D * n}});
  c.bk = grp({{(int)D, D2 * D}, {(int)D, 1}});
  c.bn = grp({{(int)d, D2 * D2}, {(int)D, D2}, {(int)D, D}});
  c.cm = grp({{(int)chi, chi * dD4}, {(int)D, 1}, {(int)chi, dD4}, {(int)D, D}});
  c.cn = grp({{(int)d, D2}, {(int)D, d * D2 * D}, {(int)D, d * D2}});
  return c;
}

// Edge renormalisation, bra layer:
// Y3[c, rk, rb, a, dk, db] = sum_{s,lb,ub} Y2[c, a, rk, dk, s, lb, ub] A[s, lb, rb, db, ub]
inline Contraction edge_bra(long long chi, long long D, long long d, long long n) {
  const long long D2 = D * D, dD4 = d * D2 * D2;
  Contraction c;
  c.am = grp({{(int)chi, chi * dD4}, {(int)chi, dD4}, {(int)D, d * D2 * D}, {(int)D, d * D2}});
  c.ak = grp({{(int)d, D2}, {(int)D, D}, {(int)D, 1}});
  c.bk = grp({{(int)d, D2 * D2}, {(int)D, D2 * D}, {(int)D, 1}});
  c.bn = grp({{(int)D, D2}, {(int)D, D}});
  c.cm = grp({{(int)chi, D2 * n}, {(int)chi, D2}, {(int)D, D * n}, {(int)D, D}});
  c.cn = grp({{(int)D, n}, {(int)D, 1}});
  return c;
}

// Edge renormalisation, step 4: T4new[e, rk, rb, c] = sum_i Y3[c, rk, rb, i] P[i, e]
inline Contraction edge_p(long long chi, long long D, long long n) {
  const long long D2 = D * D;
  Contraction c;
  c.am = grp({{(int)chi, D2 * n}, {(int)D, D * n}, {(int)D, n}});
  c.ak = grp({{(int)n, 1}});
  c.bk = grp({{(int)n, chi}});
  c.bn = grp({{(int)chi, 1}});
  c.cm = grp({{(int)chi, 1}, {(int)D, D * chi}, {(int)D, chi}});
  c.cn = grp({{(int)chi, D2 * chi}});
  return c;
}

// Half network for the reduced density matrices, bra layer with the
// physical index left open:
// X4[t][s][s'][rk][rb][e][dk][db] = sum_{lb,ub} X3[e,t,rk,dk,s,lb,ub] A[s',lb,rb,db,ub]
inline Contraction half_bra(long long chi, long long D, long long d, long long n) {
  const long long D2 = D * D, D4 = D2 * D2;
  Contraction c;
  c.am = grp({{(int)chi, chi * d * D4}, {(int)chi, d * D4}, {(int)D, d * D2 * D},
              {(int)D, d * D2}, {(int)d, D2}});
  c.ak = grp({{(int)D, D}, {(int)D, 1}});
  c.bk = grp({{(int)D, D2 * D}, {(int)D, 1}});
  c.bn = grp({{(int)d, D4}, {(int)D, D2}, {(int)D, D}});
  c.cm = grp({{(int)chi, D2}, {(int)chi, d * d * D2 * n}, {(int)D, D * n}, {(int)D, D},
              {(int)d, d * D2 * n}});
  c.cn = grp({{(int)d, D2 * n}, {(int)D, n}, {(int)D, 1}});
  return c;
}

// Half network, closing with T3 C4:
// L[(t,s,s',rk,rb), b] = sum_{e,dk,db} X4[..., e, dk, db] Y[b, dk, db, e]
inline Contraction half_close(long long chi, long long D, long long d, long long n) {
  const long long D2 = D * D;
  Contraction c;
  c.am = grp({{(int)(chi * d * d * D2), n}});
  c.ak = grp({{(int)chi, D2}, {(int)D, D}, {(int)D, 1}});
  c.bk = grp({{(int)chi, 1}, {(int)D, D * chi}, {(int)D, chi}});
  c.bn = grp({{(int)chi, D2 * chi}});
  c.cm = grp({{(int)(chi * d * d * D2), chi}});
  c.cn = grp({{(int)chi, 1}});
  return c;
}

// One-site RDM: rho1[s, s'] = sum L[t, s, s', rk, rb, b] R[t, rk, rb, b]
inline Contraction rdm_one(long long chi, long long D, long long d) {
  const long long D2 = D * D;
  Contraction c;
  c.am = grp({{(int)d, d * D2 * chi}, {(int)d, D2 * chi}});
  c.ak = grp({{(int)chi, d * d * D2 * chi}, {(int)D, D * chi}, {(int)D, chi}, {(int)chi, 1}});
  c.bk = grp({{(int)chi, D2 * chi}, {(int)D, D * chi}, {(int)D, chi}, {(int)chi, 1}});
  c.bn = grp({{1, 0}});
  c.cm = grp({{(int)d, d}, {(int)d, 1}});
  c.cn = grp({{1, 0}});
  return c;
}

// Two-site RDM from two half networks (the second one rotated by 180
// degrees): rho[(s1,s2), (s1',s2')]
inline Contraction rdm_two(long long chi, long long D, long long d) {
  const long long D2 = D * D;
  Contraction c;
  c.am = grp({{(int)d, d * D2 * chi}, {(int)d, D2 * chi}});
  c.ak = grp({{(int)chi, d * d * D2 * chi}, {(int)D, D * chi}, {(int)D, chi}, {(int)chi, 1}});
  c.bk = grp({{(int)chi, 1}, {(int)D, D * chi}, {(int)D, chi}, {(int)chi, d * d * D2 * chi}});
  c.bn = grp({{(int)d, d * D2 * chi}, {(int)d, D2 * chi}});
  c.cm = grp({{(int)d, d * d * d}, {(int)d, d}});
  c.cn = grp({{(int)d, d * d}, {(int)d, 1}});
  return c;
}

// A plain product C[M][N] = op(A) op(B) with row-major leading dimensions
// (op = transpose when ta / tb) as a contraction.
inline Contraction matmul(int M, int N, int K, long long lda, bool ta, long long ldb, bool tb,
                          long long ldc) {
  Contraction c;
  c.am = grp({{M, ta ? 1 : lda}});
  c.ak = grp({{K, ta ? lda : 1}});
  c.bk = grp({{K, tb ? 1 : ldb}});
  c.bn = grp({{N, tb ? ldb : 1}});
  c.cm = grp({{M, ldc}});
  c.cn = grp({{N, 1}});
  return c;
}

}  // namespace nets
