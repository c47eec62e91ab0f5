#include "plan_host.h"

#include <algorithm>
#include <unordered_set>

namespace pwplan {

int build_host_plan(const int32_t* miller, int64_t npw, int n1, int n2, int n3, HostPlan* out,
                    int64_t* bad_point) {
  if (!miller || !out || npw < 1 || npw > (int64_t)INT32_MAX || n1 < 1 || n2 < 1 || n3 < 1 ||
      n1 > 4096 || n2 > 4096 || n3 > 4096)
    return 2;
  HostPlan& P = *out;
  P = HostPlan();
  P.n1 = n1;
  P.n2 = n2;
  P.n3 = n3;
  P.npw = npw;
  std::vector<int> m1(npw), m2(npw), m3(npw);
  {
    std::unordered_set<int64_t> cells;
    cells.reserve((size_t)npw * 2);
    for (int64_t g = 0; g < npw; ++g) {
      const int64_t a = miller[3 * g], b = miller[3 * g + 1], c = miller[3 * g + 2];
      m1[g] = (int)(((a % n1) + n1) % n1);
      m2[g] = (int)(((b % n2) + n2) % n2);
      m3[g] = (int)(((c % n3) + n3) % n3);
      const int64_t key = ((int64_t)m3[g] * n2 + m2[g]) * n1 + m1[g];
      if (!cells.insert(key).second) {
        if (bad_point) *bad_point = g;
        return 1;
      }
    }
  }
  // points ordered by (centred m1, centred m2, centred m3): columns = runs of equal (m1, m2)
  std::vector<int>& order = P.pt_perm;
  order.resize(npw);
  for (int64_t g = 0; g < npw; ++g) order[g] = (int)g;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    const int ax = center(m1[x], n1), ay = center(m1[y], n1);
    if (ax != ay) return ax < ay;
    const int bx = center(m2[x], n2), by = center(m2[y], n2);
    if (bx != by) return bx < by;
    return center(m3[x], n3) < center(m3[y], n3);
  });
  std::vector<int> col_m1;
  P.pt_col.resize(npw);
  P.pt_m3.resize(npw);
  P.runs = 1;
  for (int64_t k = 0; k < npw; ++k) {
    const int g = order[k];
    if (k == 0 || m1[g] != m1[order[k - 1]] || m2[g] != m2[order[k - 1]]) {
      P.col_start.push_back((int)k);
      col_m1.push_back(m1[g]);
      P.col_m2.push_back(m2[g]);
      P.col_m3lo.push_back(center(m3[g], n3));
    } else if (center(m3[g], n3) != center(m3[order[k - 1]], n3) + 1) {
      P.runs = 0;   // a gap along N3 inside a column
    }
    if (g != (int)k) P.runs = 0;   // not in column order
    P.pt_col[k] = (int)P.col_start.size() - 1;
    P.pt_m3[k] = m3[g];
  }
  P.col_start.push_back((int)npw);
  P.ncols = (int)col_m1.size();
  P.ldt = (P.ncols + 15) / 16 * 16;
  // distinct m1 sorted by centred value
  P.ext_m1 = col_m1;
  std::sort(P.ext_m1.begin(), P.ext_m1.end(),
            [&](int x, int y) { return center(x, n1) < center(y, n1); });
  P.ext_m1.erase(std::unique(P.ext_m1.begin(), P.ext_m1.end()), P.ext_m1.end());
  P.xr = (int)P.ext_m1.size();
  P.quarter12 = 1;
  for (int c = 0; c < P.ncols; ++c) {
    const int a1 = center(col_m1[c], n1), a2 = center(P.col_m2[c], n2);
    if (4 * a1 < -n1 || 4 * a1 >= n1 || 4 * a2 < -n2 || 4 * a2 >= n2) P.quarter12 = 0;
  }
  std::vector<int> slot(n1, -1);
  for (int e = 0; e < P.xr; ++e) slot[P.ext_m1[e]] = e;
  P.col_e.resize(P.ncols);
  for (int c = 0; c < P.ncols; ++c) P.col_e[c] = slot[col_m1[c]];
  return 0;
}

}  // namespace pwplan
