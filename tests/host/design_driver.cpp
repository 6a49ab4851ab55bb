// Test driver of the host FP64 wavelet design of libos3d (coefficients of
// Sec. 3.2 and Eqs. 12-16, the steering matrix of Eqs. 17-19, antipodal
// pairing, the DFT radix plans), built with g++ and the address and
// undefined-behaviour sanitizers by tests/test_host_sanitizers.py.  It prints
// the coefficients for the parameter grid the test compares with the oracle,
// and checks the plans and layouts itself; any sanitizer report fails the run.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "os3d_internal.h"

using namespace os3d;

int main() {
  int bad = 0;
  const int Ls[] = {0, 1, 2, 7, 16, 24, 40, 62, 64};
  const double ss[] = {0.25, 0.7, 1.9};
  const int ks[] = {0, 2, 4};
  for (int L : Ls)
    for (double s : ss)
      for (int k : ks)
        for (int coeffs = 0; coeffs < 2; ++coeffs)
          for (int variant = 0; variant < 2; ++variant) {
            os3d_wavelet_params p = {L, s, k, 20, 0.8, 1e-3, variant, coeffs};
            std::vector<double> c, a;
            wavelet_coeffs(p, c, a);
            if ((int)c.size() != L + 1 || (int)a.size() != L + 1) ++bad;
            std::printf("coef %d %.17g %d %d %d", L, s, k, coeffs, variant);
            for (double v : a) std::printf(" %.17g", v);
            std::printf("\n");
          }
  // steering matrix and pairing on the 42-point icosahedral set
  std::vector<double> ico = geodesic_icosahedron(2);  // 42 unit vectors
  const int n = (int)ico.size() / 3;
  os3d_wavelet_params p = {24, 0.5, 2, 20, 0.8, 1e-3, OS3D_CAKE, OS3D_COEFFS_LSQ};
  std::vector<double> c, a;
  wavelet_coeffs(p, c, a);
  std::vector<double> S((size_t)25 * 25 * n);
  steering_std(p, ico.data(), n, a, S.data());
  double sum = 0.0;
  for (double v : S) sum += std::fabs(v);
  std::printf("steer %d %.17g\n", n, sum);
  std::vector<int> partner;
  pair_orientations(ico.data(), n, partner);
  for (int i = 0; i < n; ++i)
    if (partner[i] < 0 || partner[partner[i]] != i) ++bad;
  // radix plans: every supported length factors into the stages
  int plans = 0;
  for (int len = 2; len <= kMaxDim; ++len) {
    if (!factor235(len)) continue;
    std::vector<int> r = radix_schedule(len);
    long long prod = 1;
    for (int x : r) prod *= x;
    if (prod != len || (int)r.size() > kMaxStages) ++bad;
    ++plans;
  }
  // the contraction order of the bank kernel addresses every (l, m, cos / sin)
  // once (no sin entry for m = 0) within its K-blocks; the even words run
  // through the orders 0..M and the odd words through M + 1..L, each in the
  // recursion's order (l = m..L, orders ascending), and M balances the two
  for (int L : Ls) {
    const int M = synth_split(L);
    const int ne = 32 * synth_kblocks(L);
    if (ne < 2 * synth_words(L) || ne >= 2 * synth_words(L) + 32) ++bad;
    std::vector<int> seen((size_t)(L + 1) * (L + 1) * 2, 0);
    int used = 0;
    int last[2][2] = {{-1, -1}, {-1, -1}};  // per chain: previous (m, l)
    for (int e = 0; e < ne; ++e) {
      int l, m;
      bool sn;
      if (!synth_entry(L, e, l, m, sn)) continue;
      if (l < m || l > L || (m == 0 && sn)) ++bad;
      const int chain = (e >> 1) & 1;
      if ((chain == 0) != (m <= M)) ++bad;
      if (!sn) {  // steps of a chain in the recursion's order
        int* pv = last[chain];
        const bool next = (m == pv[0] && l == pv[1] + 1) || (m == pv[0] + 1 && l == m && pv[1] == L) ||
                          (pv[0] < 0 && l == m && m == (chain == 0 ? 0 : M + 1));
        if (!next) ++bad;
        pv[0] = m;
        pv[1] = l;
      }
      ++seen[(size_t)(l * (L + 1) + m) * 2 + (sn ? 1 : 0)];
      ++used;
    }
    for (int v : seen)
      if (v > 1) ++bad;
    if (used != (L + 1) * (L + 1)) ++bad;
    // the precomputed word order the host packs the operands by
    const std::vector<int> order = synth_word_order(L);
    if ((int)order.size() * 2 != ne) ++bad;
    for (int e = 0; e < ne; ++e) {
      int l, m;
      bool sn;
      const bool ok = synth_entry(L, e, l, m, sn);
      const int lm = order[e >> 1];
      const bool ok2 = lm >= 0 && !(lm % (L + 1) == 0 && (e & 1) == 1);
      if (ok != ok2 || (ok && lm != l * (L + 1) + m)) ++bad;
    }
    // balance: no other split has a shorter longer chain
    auto words = [&](int m0, int m1) {
      int n = 0;
      for (int m = m0; m <= m1; ++m) n += L + 1 - m;
      return n;
    };
    for (int M2 = 0; M2 <= L; ++M2)
      if (std::max(words(0, M2), words(M2 + 1, L)) < synth_pairs(L)) ++bad;
  }
  std::printf("plans %d bad %d\n", plans, bad);
  return bad ? 1 : 0;
}
