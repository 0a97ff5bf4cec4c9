// Host-only driver for the sanitized build of the reference-element tables:
// builds them for every displacement/pressure order pair and prints the sums
// of the mass tables (the reference tetrahedron's volume) and the element
// Jacobi bounds, which the calling test compares with their known values.
#include <cstdio>
#include <vector>

#include "nm_internal.h"

int main() {
  for (int du = 1; du <= 2; ++du)
    for (int dp = 1; dp <= 2; ++dp) {
      nm::RefTables t;
      nm::build_ref_tables(du, dp, t);
      double s = 0.0, sp = 0.0;
      for (int a = 0; a < t.nd; ++a)
        for (int b = 0; b < t.nd; ++b) s += t.MM[a][b];
      for (int a = 0; a < t.npp; ++a)
        for (int b = 0; b < t.npp; ++b) sp += t.Mp[a][b];
      std::printf("orders %d %d: nd %d npp %d mass sum %.15g pressure mass sum %.15g bounds %.6g %.6g %.6g %.6g\n",
                  du, dp, t.nd, t.npp, s, sp, t.m_lo, t.m_hi, t.p_lo, t.p_hi);
    }
  std::vector<double> a = {2.0, 1.0, 1.0, 2.0}, w, v;
  nm::jacobi_eig(2, a, w, &v);
  std::printf("jacobi %.15g %.15g\n", w[0], w[1]);
  return 0;
}
