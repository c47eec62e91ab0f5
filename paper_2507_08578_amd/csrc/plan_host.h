// Sphere -> box maps of one Hamiltonian, built on the host (plain C++, no GPU
// code) once per handle and uploaded as the device arrays of BoxPlan.  The
// layout they describe is the pruned FFT route's: sphere points grouped into
// columns along N3 (equal (m1, m2)), columns ordered by centred (m1, m2),
// points within a column by centred m3, and the extent of distinct m1.
#pragma once

#include <cstdint>
#include <vector>

namespace pwplan {

// centred index of box index m in [0, n): m for m <= n/2, else m - n
inline int center(int m, int n) { return m <= n / 2 ? m : m - n; }

struct HostPlan {
  int n1 = 0, n2 = 0, n3 = 0;
  int64_t npw = 0;
  int ncols = 0;       // distinct (m1, m2)
  int ldt = 0;         // ncols rounded up to a multiple of 16
  int xr = 0;          // distinct m1
  int quarter12 = 0;   // every centred m1 in [-n1/4, n1/4) and m2 in [-n2/4, n2/4)
  int runs = 0;        // caller order is column order and every column is gap-free along N3
  std::vector<int> col_start;   // ncols + 1: first point (column order) of each column
  std::vector<int> col_e;       // ncols: extent slot of the column's m1
  std::vector<int> col_m2;      // ncols: box index m2
  std::vector<int> col_m3lo;    // ncols: centred m3 of the column's first point
  std::vector<int> pt_perm;     // npw: caller index of the k-th point in column order
  std::vector<int> pt_col;      // npw: column of the k-th point
  std::vector<int> pt_m3;       // npw: box index m3 of the k-th point
  std::vector<int> ext_m1;      // xr: box index m1 of extent slot e, by centred m1
};

// miller: npw x 3 int32 triples, row-major (any sign; reduced modulo the box).  Box
// lengths in [1, 4096], npw in [1, 2^31).  Returns 0 and fills *out, or
// returns 1 with *bad_point = the first point whose box cell an earlier
// point already holds (the box is too small for the sphere), or 2 for
// arguments out of range.
int build_host_plan(const int32_t* miller, int64_t npw, int n1, int n2, int n3, HostPlan* out,
                    int64_t* bad_point);

}  // namespace pwplan
