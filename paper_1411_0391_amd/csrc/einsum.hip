// Pairwise tensor contraction by index labels, mapped onto the table-driven
// MFMA contraction engine: "xlLg,gh->xlLh" contracts the labels shared by the
// two operands and absent from the output.  Labels in the output come from
// exactly one operand (no batch labels, no traces); the output is row-major
// in the order the spec lists.  Adjacent labels that are contiguous in every
// operand they appear in are merged, so plain matrix products run on the
// strided path.
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "common.h"

namespace {

struct Lab {
  char c;
  int ext;
  long long s1, s2;  // strides in the two operands the group pairs
};

// The groups of one kind of label in the two operands it pairs (A and C for
// the free labels of A, B and C for those of B, A and B for the contracted
// ones); neighbours that walk both operands contiguously are merged.
void merged(const std::vector<Lab>& v, IdxGroup* g1, IdxGroup* g2) {
  std::vector<Lab> m;
  for (const Lab& l : v) {
    if (l.ext == 1) continue;  // extent-1 labels carry no offset
    if (!m.empty()) {
      Lab& p = m.back();
      if (p.s1 == (long long)l.ext * l.s1 && p.s2 == (long long)l.ext * l.s2) {
        p.ext *= l.ext;
        p.s1 = l.s1;
        p.s2 = l.s2;
        continue;
      }
    }
    m.push_back(l);
  }
  *g1 = IdxGroup();
  *g2 = IdxGroup();
  for (const Lab& l : m) {
    g1->ext.push_back(l.ext);
    g1->str.push_back(l.s1);
    g2->ext.push_back(l.ext);
    g2->str.push_back(l.s2);
  }
  if (m.empty()) {  // a group of no labels is one element at offset 0
    g1->ext.push_back(1);
    g1->str.push_back(0);
    g2->ext.push_back(1);
    g2->str.push_back(0);
  }
}

}  // namespace

int ein(tn_ctx* ctx, const char* spec, const double* A, std::initializer_list<int> da,
        const double* B, std::initializer_list<int> db, double* C, double alpha, double beta,
        int prec) {
  const char* comma = std::strchr(spec, ',');
  const char* arrow = std::strstr(spec, "->");
  if (!comma || !arrow || arrow < comma) TN_FAIL(ctx, TN_EINVAL, "bad contraction spec %s", spec);
  const std::string sa(spec, comma), sb(comma + 1, arrow), sc(arrow + 2);
  const std::vector<int> va(da), vb(db);
  if (sa.size() != va.size() || sb.size() != vb.size())
    TN_FAIL(ctx, TN_EINVAL, "contraction %s: rank and extents disagree", spec);
  std::map<char, int> ext;
  std::map<char, long long> stA, stB, stC;
  auto strides = [&](const std::string& s, const std::vector<int>& d,
                     std::map<char, long long>& st) -> int {
    long long acc = 1;
    for (int i = (int)s.size() - 1; i >= 0; --i) {
      if (st.count(s[i])) TN_FAIL(ctx, TN_EINVAL, "contraction %s: repeated label", spec);
      st[s[i]] = acc;
      acc *= d[i];
      auto it = ext.find(s[i]);
      if (it != ext.end() && it->second != d[i])
        TN_FAIL(ctx, TN_EINVAL, "contraction %s: label %c has extents %d and %d", spec, s[i],
                it->second, d[i]);
      ext[s[i]] = d[i];
    }
    return TN_OK;
  };
  TN_TRY(strides(sa, va, stA));
  TN_TRY(strides(sb, vb, stB));
  {
    long long acc = 1;
    for (int i = (int)sc.size() - 1; i >= 0; --i) {
      if (!ext.count(sc[i])) TN_FAIL(ctx, TN_EINVAL, "contraction %s: unknown output label", spec);
      if (stC.count(sc[i])) TN_FAIL(ctx, TN_EINVAL, "contraction %s: repeated label", spec);
      stC[sc[i]] = acc;
      acc *= ext[sc[i]];
    }
  }
  std::vector<Lab> m, n, k;
  for (char c : sc) {
    const bool inA = stA.count(c), inB = stB.count(c);
    if (inA && inB) TN_FAIL(ctx, TN_EINVAL, "contraction %s: batch labels unsupported", spec);
    if (inA) m.push_back({c, ext[c], stA[c], stC[c]});
    else n.push_back({c, ext[c], stB[c], stC[c]});
  }
  for (char c : sa) {
    if (stC.count(c)) continue;
    if (!stB.count(c)) TN_FAIL(ctx, TN_EINVAL, "contraction %s: label %c only in A", spec, c);
    k.push_back({c, ext[c], stA[c], stB[c]});
  }
  for (char c : sb)
    if (!stC.count(c) && !stA.count(c))
      TN_FAIL(ctx, TN_EINVAL, "contraction %s: label %c only in B", spec, c);
  Contraction ct;
  merged(m, &ct.am, &ct.cm);
  merged(n, &ct.bn, &ct.cn);
  merged(k, &ct.ak, &ct.bk);
  return tc_run(ctx, ct, A, B, C, alpha, beta, prec);
}
