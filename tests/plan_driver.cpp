// Test driver for the host-side sphere -> box map builder: reads
// "n1 n2 n3 npw" and npw Miller triples from stdin, prints the return code,
// the offending point, the scalar fields and every array, one per line.
#include <cstdio>
#include <vector>

#include "plan_host.h"

static void put(const char* name, const std::vector<int>& v) {
  std::printf("%s", name);
  for (int x : v) std::printf(" %d", x);
  std::printf("\n");
}

int main() {
  int n1, n2, n3;
  long long npw;
  if (std::scanf("%d %d %d %lld", &n1, &n2, &n3, &npw) != 4) return 3;
  std::vector<int32_t> miller((size_t)(npw > 0 ? npw : 0) * 3);
  for (auto& m : miller)
    if (std::scanf("%d", &m) != 1) return 3;
  pwplan::HostPlan p;
  int64_t bad = -1;
  const int rc = pwplan::build_host_plan(miller.empty() ? nullptr : miller.data(), npw, n1, n2,
                                         n3, &p, &bad);
  std::printf("rc %d\nbad %lld\n", rc, (long long)bad);
  if (rc != 0) return 0;
  std::printf("scalars %d %d %d %d %d\n", p.ncols, p.ldt, p.xr, p.quarter12, p.runs);
  put("col_start", p.col_start);
  put("col_e", p.col_e);
  put("col_m2", p.col_m2);
  put("col_m3lo", p.col_m3lo);
  put("pt_perm", p.pt_perm);
  put("pt_col", p.pt_col);
  put("pt_m3", p.pt_m3);
  put("ext_m1", p.ext_m1);
  return 0;
}
