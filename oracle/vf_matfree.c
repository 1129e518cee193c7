/* Matrix-free FP64 product with the centroid-rule view factors of eq. (10)
 * (oracle; TEST INFRASTRUCTURE ONLY: loaded by oracle/matfree.py, which only
 * tests/, the smoke check and the bench's CPU baseline use; nothing of the
 * library links or calls it).
 *
 * Y = F X for n facets without storing F: every entry is evaluated when it is
 * used, with the same readings and the same operation order as
 * oracle/viewfactor.py (per-area convention F_ij = cos_i cos_j A_j / (pi r^2),
 * back-facing pairs and coincident centroids give 0, F_ii = 0), so each
 * entry equals the dense oracle's bit for bit:
 *   d = c_j - c_i;  r2 = (dx*dx + dy*dy) + dz*dz;
 *   ci = (nix*dx + niy*dy) + niz*dz;  cj = -((njx*dx + njy*dy) + njz*dz);
 *   F = (max(ci,0) * max(cj,0) * A_j) / ((pi * r2) * r2).
 * Row i of Y is summed over j = 0, 1, ..., n-1 in that order.  Eight rows
 * are evaluated side by side (one SIMD lane each); rows are shared among
 * OpenMP threads.  Build: gcc -O2 -fopenmp -ffp-contract=off (no fused
 * multiply-add, no reassociation).
 *
 * Layout: coordinates and normals as separate x, y, z arrays of n; X and Y
 * row-major n x r (the r values of one facet contiguous), 1 <= r <= 16.
 */
#include <stdint.h>

#define LANES 8
#define MAXR 16

static const double PI = 3.14159265358979323846;

void vf_matvec(int64_t n, const double* cx, const double* cy, const double* cz, const double* nx, const double* ny,
               const double* nz, const double* area, int64_t r, const double* X, double* Y) {
  if (r < 1 || r > MAXR) return;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i0 = 0; i0 < n; i0 += LANES) {
    double acc[MAXR][LANES];
    double pix[LANES], piy[LANES], piz[LANES], nix[LANES], niy[LANES], niz[LANES];
    int64_t idx[LANES];
    for (int l = 0; l < LANES; ++l) {
      const int64_t i = i0 + l < n ? i0 + l : n - 1;
      idx[l] = i0 + l;
      pix[l] = cx[i];
      piy[l] = cy[i];
      piz[l] = cz[i];
      nix[l] = nx[i];
      niy[l] = ny[i];
      niz[l] = nz[i];
      for (int q = 0; q < MAXR; ++q) acc[q][l] = 0.0;
    }
    for (int64_t j = 0; j < n; ++j) {
      const double qx = cx[j], qy = cy[j], qz = cz[j];
      const double mx = nx[j], my = ny[j], mz = nz[j], aj = area[j];
      double f[LANES];
#pragma omp simd
      for (int l = 0; l < LANES; ++l) {
        const double dx = qx - pix[l], dy = qy - piy[l], dz = qz - piz[l];
        const double r2 = (dx * dx + dy * dy) + dz * dz;
        const double ci = (nix[l] * dx + niy[l] * dy) + niz[l] * dz;
        const double cj = -((mx * dx + my * dy) + mz * dz);
        const double num = (ci > 0.0 ? ci : 0.0) * (cj > 0.0 ? cj : 0.0) * aj;
        const double den = (PI * r2) * r2;
        const double v = num / den;
        f[l] = (r2 > 0.0 && idx[l] != j) ? v : 0.0;
      }
      const double* xj = X + j * r;
      for (int64_t q = 0; q < r; ++q) {
        const double xv = xj[q];
#pragma omp simd
        for (int l = 0; l < LANES; ++l) acc[q][l] += f[l] * xv;
      }
    }
    for (int l = 0; l < LANES; ++l) {
      if (i0 + l >= n) break;
      for (int64_t q = 0; q < r; ++q) Y[(i0 + l) * r + q] = acc[q][l];
    }
  }
}
