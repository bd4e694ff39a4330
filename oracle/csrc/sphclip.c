/* Oracle helper (test infrastructure only): area of the intersection of two convex spherical
 * polygons on the unit sphere.
 *
 * Sec. 4.1 of the paper computes the areas A_km shared by a coarse hexagon k and a fine
 * hexagon m.  Here the intersection is found with the Sutherland-Hodgman algorithm, clipping
 * the subject polygon against the great-circle half-spaces of the clip polygon's edges, and its
 * area is the sum of a fan of spherical triangles (Van Oosterom-Strackee formula).
 * Both polygons are given counter-clockwise seen from outside and are smaller than a
 * hemisphere.  Plain loops, double precision. */
#include <math.h>

#define MAXV 32

static void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static double tri_area(const double* a, const double* b, const double* c) {
  double bc[3];
  cross3(b, c, bc);
  double num = dot3(a, bc);
  double den = 1.0 + dot3(a, b) + dot3(b, c) + dot3(c, a);
  return 2.0 * atan2(num, den);
}

/* clip polygon (in, n) by half-space {x : x . nrm >= 0}; returns new vertex count */
static int clip_half(const double in[][3], int n, const double* nrm, double out[][3]) {
  int m = 0;
  for (int i = 0; i < n; ++i) {
    const double* s = in[i];
    const double* e = in[(i + 1) % n];
    double ds = dot3(s, nrm), de = dot3(e, nrm);
    int s_in = ds >= 0.0, e_in = de >= 0.0;
    if (s_in && m < MAXV) {
      out[m][0] = s[0]; out[m][1] = s[1]; out[m][2] = s[2]; ++m;
    }
    if (s_in != e_in && m < MAXV) {
      /* point of the arc s-e on the great circle: positive combination of s and e */
      double a = fabs(de), b = fabs(ds);
      double x[3] = {a * s[0] + b * e[0], a * s[1] + b * e[1], a * s[2] + b * e[2]};
      double r = sqrt(dot3(x, x));
      out[m][0] = x[0] / r; out[m][1] = x[1] / r; out[m][2] = x[2] / r; ++m;
    }
  }
  return m;
}

double sph_overlap_area(const double* P, int np, const double* Q, int nq) {
  double A[MAXV][3], B[MAXV][3];
  int n = np;
  for (int i = 0; i < np; ++i)
    for (int k = 0; k < 3; ++k) A[i][k] = P[3 * i + k];
  for (int j = 0; j < nq && n > 0; ++j) {
    double nrm[3];
    cross3(&Q[3 * j], &Q[3 * ((j + 1) % nq)], nrm);
    n = clip_half((const double(*)[3])A, n, nrm, B);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < 3; ++k) A[i][k] = B[i][k];
  }
  if (n < 3) return 0.0;
  double area = 0.0;
  for (int i = 1; i + 1 < n; ++i) area += tri_area(A[0], A[i], A[i + 1]);
  return area;
}

/* batch form: pairs k = 0..npairs-1, polygons padded to 6 vertices */
void sph_overlap_areas(int npairs, const double* P, const int* np, const double* Q, const int* nq,
                       double* out) {
  for (int k = 0; k < npairs; ++k) out[k] = sph_overlap_area(P + 18 * k, np[k], Q + 18 * k, nq[k]);
}
