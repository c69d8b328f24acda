// Storage of a symmetric element operator of the GD basis (host and device).
//
// In 1D two GD functions of degree p interact iff their nodes are at most p apart
// (bandwidth p, Sec. 3.1).  In 2D row i = (ix, iy) of an element matrix therefore
// couples with columns (jx, jy), |jx - ix| <= p, |jy - iy| <= p, inside the element.
// Only the upper half in the flat order i = iy*(N+1) + ix is stored:
//   U(i) = {(jx, iy) : ix <= jx <= xhi(ix)}  followed by
//          {(jx, jy) : iy < jy <= min(iy+p, N), xlo(ix) <= jx <= xhi(ix)}   (row-major)
// with xlo(k) = max(k - p, 0), xhi(k) = min(k + p, N).  rowoff[i] is the start of
// row i's upper part; the total is (sum_k w(k))^2 / 2 + (N+1)^2 / 2 entries.
#pragma once

#ifdef __HIPCC__
#define GDW_HD __host__ __device__
#else
#define GDW_HD
#endif

namespace gdw {

GDW_HD inline int st_lo(int k, int p) { return k - p > 0 ? k - p : 0; }
GDW_HD inline int st_hi(int k, int p, int N) { return k + p < N ? k + p : N; }
GDW_HD inline int st_w(int k, int p, int N) { return st_hi(k, p, N) - st_lo(k, p) + 1; }

// number of stored entries of row (ix, iy)
GDW_HD inline int st_count(int ix, int iy, int p, int N) {
  const int same = st_hi(ix, p, N) - ix + 1;
  const int above = st_hi(iy, p, N) - iy;
  return same + above * st_w(ix, p, N);
}

// position, relative to rowoff of row (ix, iy), of column (jx, jy) in U(ix, iy);
// requires (jx, jy) in U(ix, iy)
GDW_HD inline int st_pos(int ix, int iy, int jx, int jy, int p, int N) {
  if (jy == iy) return jx - ix;
  return (st_hi(ix, p, N) - ix + 1) + (jy - iy - 1) * st_w(ix, p, N) + (jx - st_lo(ix, p));
}

// is (jx, jy) stored in the upper part of row (ix, iy)?
GDW_HD inline bool st_in_upper(int ix, int iy, int jx, int jy, int p, int N) {
  if (jy == iy) return jx >= ix && jx <= st_hi(ix, p, N);
  return jy > iy && jy <= st_hi(iy, p, N) && jx >= st_lo(ix, p) && jx <= st_hi(ix, p, N);
}

}  // namespace gdw
