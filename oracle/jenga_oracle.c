/*
 * FP64 CPU oracle for batched stepping of towers of oriented boxes.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg.  It shares no code with the HIP library.
 *
 * One step of a tower, in the order the paper describes it (Secs. "Rigid-Body
 * Foundations", "Physics Engine --- Collision Detection", "Contact Solver ---
 * Projected Gauss-Seidel (PGS)"), with the readings of unclear passages listed
 * in the design notes:
 *   1. external forces: v += dt g + dt F/m  (semi-implicit Euler, gravity first)
 *   2. frames: R(q) by Eq. (rotmat), world AABB, I_w^-1 = R I_b^-1 R^T
 *   3. broadphase: Eq. (aabb) with epsilon = 2 mm on all pairs, plus the ground
 *   4. narrowphase: 15-axis SAT, normal = axis of least penetration
 *   5. manifold: project corners, convex hulls, Sutherland-Hodgman clip, <= 4 samples
 *   6. colouring: greedy first fit over manifolds in canonical (a, b) order
 *   7. prep: r_A, r_B and inverse effective masses, Eq. (keff)
 *   8. PGS: Eq. (lambda_n) and Eq. (coulomb_pgs), colour by colour
 *   9. residual of the solve (natural map)
 *  10. integrate: x += dt v, Eq. (quat_int) with world-frame omega, angular
 *      momentum carried across the rotation (Eq. (newton_euler), torque free)
 *  11. Baumgarte position correction, Eq. (baumgarte)
 */
#include "jenga_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAX_COLOURS 64
#define CROSS_SKIP 1e-5      /* cross axes shorter than this are not tested */
#define MERGE_DIST 1e-6      /* clip vertices closer than this are merged */
#define BAND 1e-6            /* precision band width [m] */
#define HULL_EPS 1e-15       /* turn threshold of the convex hull [m^2] */

/* ------------------------------------------------------------------------------------------ */
/* small vector helpers                                                                        */
/* ------------------------------------------------------------------------------------------ */

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double a[3], const double b[3], double c[3]) {
  double x = a[1] * b[2] - a[2] * b[1];
  double y = a[2] * b[0] - a[0] * b[2];
  double z = a[0] * b[1] - a[1] * b[0];
  c[0] = x; c[1] = y; c[2] = z;
}

static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }

static void mat_vec(const double M[9], const double a[3], double c[3]) {
  double x = M[0] * a[0] + M[1] * a[1] + M[2] * a[2];
  double y = M[3] * a[0] + M[4] * a[1] + M[5] * a[2];
  double z = M[6] * a[0] + M[7] * a[1] + M[8] * a[2];
  c[0] = x; c[1] = y; c[2] = z;
}

/* column i of a row-major 3x3 matrix: body axis i in world coordinates */
static void col3(const double R[9], int i, double c[3]) { c[0] = R[i]; c[1] = R[3 + i]; c[2] = R[6 + i]; }

/* M = R diag(d) R^T */
static void rot_diag_rotT(const double R[9], const double d[3], double M[9]) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += R[3 * r + k] * d[k] * R[3 * c + k];
      M[3 * r + c] = s;
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Eq. (rotmat), Eq. (inertia)                                                                 */
/* ------------------------------------------------------------------------------------------ */

void or_quat_to_rot(const double q[4], double R[9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - z * w);       R[2] = 2.0 * (x * z + y * w);
  R[3] = 2.0 * (x * y + z * w);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - x * w);
  R[6] = 2.0 * (x * z - y * w);       R[7] = 2.0 * (y * z + x * w);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

void or_box_inertia(double m, const double he[3], double I[3]) {
  /* l x w x h = full sizes along body x, y, z */
  const double l = 2.0 * he[0], wd = 2.0 * he[1], h = 2.0 * he[2];
  I[0] = m / 12.0 * (wd * wd + h * h);
  I[1] = m / 12.0 * (l * l + h * h);
  I[2] = m / 12.0 * (l * l + wd * wd);
}

static void box_corner(const double he[3], const double x[3], const double R[9], int k, double p[3]) {
  double s[3] = {(k & 1) ? he[0] : -he[0], (k & 2) ? he[1] : -he[1], (k & 4) ? he[2] : -he[2]};
  double r[3];
  mat_vec(R, s, r);
  p[0] = x[0] + r[0]; p[1] = x[1] + r[1]; p[2] = x[2] + r[2];
}

/* ------------------------------------------------------------------------------------------ */
/* SAT (Sec. "Narrowphase: OBB SAT")                                                           */
/* ------------------------------------------------------------------------------------------ */

/* prefer_face (reference-face manifolds, reading of the usual box-box clipping): a colliding pair
 * takes its normal and depth from the best face axis (first strict minimum over A0..B2) unless the
 * best axis overall is a cross axis whose overlap is below 0.95 of the face axis's by more than
 * 1e-6 m; a cross axis parallel to a face normal then never stands in for the face. */
static void sat_R(const double heA[3], const double xA[3], const double RA[9],
                  const double heB[3], const double xB[3], const double RB[9], int prefer_face,
                  or_sat_result* out) {
  double A[3][3], B[3][3], d[3];
  for (int i = 0; i < 3; ++i) { col3(RA, i, A[i]); col3(RB, i, B[i]); }
  for (int k = 0; k < 3; ++k) d[k] = xB[k] - xA[k];

  double axes[15][3];
  double delta[15];
  int tested[15];
  int band = 0;
  for (int i = 0; i < 3; ++i) { memcpy(axes[i], A[i], sizeof(double) * 3); memcpy(axes[3 + i], B[i], sizeof(double) * 3); }
  for (int i = 0; i < 6; ++i) tested[i] = 1;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      int a = 6 + 3 * i + j;
      double c[3];
      cross3(A[i], B[j], c);
      double len = norm3(c);
      if (len >= 0.9 * CROSS_SKIP && len <= 1.1 * CROSS_SKIP) band |= OR_BAND_CROSS;
      if (len < CROSS_SKIP) { tested[a] = 0; continue; }
      tested[a] = 1;
      for (int k = 0; k < 3; ++k) axes[a][k] = c[k] / len;
    }
  int best = -1;
  for (int a = 0; a < 15; ++a) {
    if (!tested[a]) continue;
    const double* u = axes[a];
    double rA = 0.0, rB = 0.0;
    for (int i = 0; i < 3; ++i) { rA += heA[i] * fabs(dot3(A[i], u)); rB += heB[i] * fabs(dot3(B[i], u)); }
    delta[a] = rA + rB - fabs(dot3(d, u));
    if (best < 0 || delta[a] < delta[best]) best = a;   /* first strict minimum */
  }
  double dmin = delta[best];
  const double dsep = dmin;   /* the separation test takes the smallest overlap of all axes */
  int rivals = 15;            /* axes that compete with the chosen one */
  out->collide = dmin > 0.0;
  if (prefer_face && best < 6) rivals = 6;
  if (prefer_face && best >= 6 && dmin > 0.0) {
    int f = 0;
    for (int a = 1; a < 6; ++a)
      if (delta[a] < delta[f]) f = a;
    const double cut = 0.95 * delta[f] - 1e-6;
    if (fabs(dmin - cut) < BAND) band |= OR_BAND_NORMAL;   /* the choice sits at its threshold */
    if (!(dmin < cut)) {
      best = f;
      dmin = delta[f];
      rivals = 6;
    }
  }
  out->axis = best;
  out->depth = dmin;
  out->sigma = -dsep;
  double s = dot3(d, axes[best]) < 0.0 ? -1.0 : 1.0;
  for (int k = 0; k < 3; ++k) out->normal[k] = s * axes[best][k];
  if (fabs(out->sigma) < BAND) band |= OR_BAND_SEPARATION;
  /* second best axis that is not parallel to the chosen one (axes closer than ~4e-7 rad give
   * the same normal to single precision; anything further apart changes the contact frame) */
  for (int a = 0; a < rivals; ++a) {
    if (!tested[a] || a == best) continue;
    if (fabs(dot3(axes[a], axes[best])) > 1.0 - 1e-13) continue;
    if (delta[a] - dmin < BAND) band |= OR_BAND_NORMAL;
  }
  out->band = band;
}

void or_sat(const double heA[3], const double xA[3], const double qA[4],
            const double heB[3], const double xB[3], const double qB[4], or_sat_result* out) {
  double RA[9], RB[9];
  or_quat_to_rot(qA, RA);
  or_quat_to_rot(qB, RB);
  sat_R(heA, xA, RA, heB, xB, RB, 0, out);
}

void or_sat_ex(const double heA[3], const double xA[3], const double qA[4],
               const double heB[3], const double xB[3], const double qB[4], int32_t prefer_face,
               or_sat_result* out) {
  double RA[9], RB[9];
  or_quat_to_rot(qA, RA);
  or_quat_to_rot(qB, RB);
  sat_R(heA, xA, RA, heB, xB, RB, prefer_face != 0, out);
}

/* ------------------------------------------------------------------------------------------ */
/* Manifold (Sec. "Contact Manifold (Face Clipping)")                                           */
/* ------------------------------------------------------------------------------------------ */

typedef struct { double u, v; } pt2;

static double cross2(pt2 o, pt2 a, pt2 b) { return (a.u - o.u) * (b.v - o.v) - (a.v - o.v) * (b.u - o.u); }

static int cmp_pt2(const void* pa, const void* pb) {
  const pt2* a = (const pt2*)pa;
  const pt2* b = (const pt2*)pb;
  if (a->u < b->u) return -1;
  if (a->u > b->u) return 1;
  if (a->v < b->v) return -1;
  if (a->v > b->v) return 1;
  return 0;
}

/* Convex hull, counter-clockwise, collinear and repeated points dropped (the hull is a
 * set: any hull algorithm, QuickHull included, returns these vertices). Returns count.
 * Corners that project onto the same point (a box seen along one of its axes shows each
 * corner of the silhouette twice, equal up to rounding) count once: points within 1e-12 m
 * of an earlier point are removed before the chain is built. */
static int convex_hull(pt2* p, int n, pt2* h) {
  int nd = 0;
  for (int i = 0; i < n; ++i) {
    int dup = 0;
    for (int j = 0; j < nd; ++j)
      if (hypot(p[i].u - p[j].u, p[i].v - p[j].v) < 1e-12) { dup = 1; break; }
    if (!dup) p[nd++] = p[i];
  }
  n = nd;
  qsort(p, (size_t)n, sizeof(pt2), cmp_pt2);
  int k = 0;
  for (int i = 0; i < n; ++i) {                       /* lower chain */
    while (k >= 2 && cross2(h[k - 2], h[k - 1], p[i]) <= HULL_EPS) --k;
    h[k++] = p[i];
  }
  for (int i = n - 2, lo = k + 1; i >= 0; --i) {      /* upper chain */
    while (k >= lo && cross2(h[k - 2], h[k - 1], p[i]) <= HULL_EPS) --k;
    h[k++] = p[i];
  }
  --k;   /* last point repeats the first */
  /* drop vertices that coincide with their predecessor */
  int m = 0;
  for (int i = 0; i < k; ++i) {
    if (m > 0 && hypot(h[i].u - h[m - 1].u, h[i].v - h[m - 1].v) < 1e-12) continue;
    h[m++] = h[i];
  }
  while (m > 1 && hypot(h[m - 1].u - h[0].u, h[m - 1].v - h[0].v) < 1e-12) --m;
  return m;
}

/* Sutherland-Hodgman: clip polygon `sub` (ns vertices) by every edge of the convex CCW
 * polygon `clip` (nc vertices).  Keeps the side left of each clip edge. */
static int sutherland_hodgman(const pt2* sub, int ns, const pt2* clip, int nc, pt2* out) {
  pt2 buf_a[64], buf_b[64];
  int n = ns;
  memcpy(buf_a, sub, sizeof(pt2) * (size_t)ns);
  pt2* in = buf_a;
  pt2* res = buf_b;
  for (int e = 0; e < nc && n > 0; ++e) {
    pt2 e0 = clip[e], e1 = clip[(e + 1) % nc];
    int m = 0;
    for (int i = 0; i < n; ++i) {
      pt2 s = in[(i + n - 1) % n], t = in[i];
      double fs = cross2(e0, e1, s), ft = cross2(e0, e1, t);
      int s_in = fs >= 0.0, t_in = ft >= 0.0;
      if (t_in) {
        if (!s_in) {
          double a = fs / (fs - ft);
          res[m].u = s.u + a * (t.u - s.u); res[m].v = s.v + a * (t.v - s.v); ++m;
        }
        res[m++] = t;
      } else if (s_in) {
        double a = fs / (fs - ft);
        res[m].u = s.u + a * (t.u - s.u); res[m].v = s.v + a * (t.v - s.v); ++m;
      }
    }
    n = m;
    pt2* tmp = in; in = res; res = tmp;
  }
  memcpy(out, in, sizeof(pt2) * (size_t)n);
  return n;
}

/* Tangent basis of a contact normal: t1 from world x (or world y when n is close to x). */
static void tangent_basis(const double n[3], double t1[3], double t2[3]) {
  double e[3] = {0.0, 0.0, 0.0};
  if (fabs(n[0]) < 0.9) e[0] = 1.0; else e[1] = 1.0;
  double en = dot3(e, n);
  for (int k = 0; k < 3; ++k) t1[k] = e[k] - en * n[k];
  double l = norm3(t1);
  for (int k = 0; k < 3; ++k) t1[k] /= l;
  cross3(n, t1, t2);
}

static int manifold_box_R(const double heA[3], const double xA[3], const double RA[9],
                          const double heB[3], const double xB[3], const double RB[9],
                          const double n[3], double depth, or_manifold* m) {
  double t1[3], t2[3];
  tangent_basis(n, t1, t2);
  memcpy(m->normal, n, sizeof(double) * 3);
  memcpy(m->t1, t1, sizeof(double) * 3);
  memcpy(m->t2, t2, sizeof(double) * 3);
  m->depth = depth;

  /* a) project the 8 corners of each box onto the plane normal to n */
  pt2 pa[8], pb[8];
  double cA[8][3], cB[8][3];
  double zA = -INFINITY, zB = INFINITY;
  int supA = 0, supB = 0;
  for (int k = 0; k < 8; ++k) {
    box_corner(heA, xA, RA, k, cA[k]);
    box_corner(heB, xB, RB, k, cB[k]);
    pa[k].u = dot3(cA[k], t1); pa[k].v = dot3(cA[k], t2);
    pb[k].u = dot3(cB[k], t1); pb[k].v = dot3(cB[k], t2);
    double da = dot3(cA[k], n), db = dot3(cB[k], n);
    if (da > zA) { zA = da; supA = k; }
    if (db < zB) { zB = db; supB = k; }
  }
  /* b) convex hulls */
  pt2 ha[16], hb[16];
  int na = convex_hull(pa, 8, ha);
  int nb = convex_hull(pb, 8, hb);
  /* c) clip A's polygon by B's */
  pt2 poly[64];
  int np = sutherland_hodgman(ha, na, hb, nb, poly);
  /* merge consecutive vertices closer than MERGE_DIST */
  pt2 mg[64];
  int nm = 0;
  for (int i = 0; i < np; ++i) {
    if (nm > 0) {
      double dd = hypot(poly[i].u - mg[nm - 1].u, poly[i].v - mg[nm - 1].v);
      if (dd > 0.9 * MERGE_DIST && dd < 1.1 * MERGE_DIST) m->band |= OR_BAND_CLIP;
      if (dd < MERGE_DIST) continue;
    }
    mg[nm++] = poly[i];
  }
  while (nm > 1) {
    double dd = hypot(mg[nm - 1].u - mg[0].u, mg[nm - 1].v - mg[0].v);
    if (dd > 0.9 * MERGE_DIST && dd < 1.1 * MERGE_DIST) m->band |= OR_BAND_CLIP;
    if (dd < MERGE_DIST) --nm; else break;
  }
  const double zmid = 0.5 * (zA + zB);
  m->npts = 0;
  if (nm == 0) {
    /* empty clip: one point halfway between the two support corners */
    for (int k = 0; k < 3; ++k) m->point[0][k] = 0.5 * (cA[supA][k] + cB[supB][k]);
    m->slot[0] = 0;
    m->npts = 1;
    m->band |= OR_BAND_EMPTY;
    return 1;
  }
  /* d) sample up to 4 points: the vertices extreme along the diagonals of (t1, t2) */
  static const double diag[4][2] = {{1.0, 1.0}, {-1.0, 1.0}, {-1.0, -1.0}, {1.0, -1.0}};
  int chosen[4];
  int nchosen = 0;
  for (int s = 0; s < 4; ++s) {
    int best = 0;
    double bv = diag[s][0] * mg[0].u + diag[s][1] * mg[0].v;
    for (int i = 1; i < nm; ++i) {
      double val = diag[s][0] * mg[i].u + diag[s][1] * mg[i].v;
      if (val > bv) { bv = val; best = i; }
    }
    for (int i = 0; i < nm; ++i) {
      if (i == best) continue;
      double val = diag[s][0] * mg[i].u + diag[s][1] * mg[i].v;
      if (bv - val < BAND) m->band |= OR_BAND_CLIP;
    }
    int dup = 0;
    for (int c = 0; c < nchosen; ++c) dup |= (chosen[c] == best);
    if (dup) continue;
    chosen[nchosen++] = best;
    /* lift to the mid-plane of the overlap slab */
    int j = m->npts++;
    for (int k = 0; k < 3; ++k) m->point[j][k] = mg[best].u * t1[k] + mg[best].v * t2[k] + zmid * n[k];
    m->slot[j] = s;
  }
  return 1;
}

/* Reference-face clipping (the alternative to the literal silhouettes): for a face axis the face
 * of the box that owns it is the reference face (outward normal u: +n for a face of A, -n for a
 * face of B); the other box's face most opposed to u is the incident face.  The incident face's
 * quad is clipped by the reference face's four side planes (Sutherland-Hodgman in 3-D); of the
 * clipped vertices those on or below the reference face (separation s >= 0 along u) are kept, and
 * each point sits halfway between its vertex and the reference face (v + s u / 2).  The up to four
 * samples are the kept vertices extreme along the diagonals of (t1, t2), as for the silhouettes.
 * An edge-edge axis gives one point: the midpoint of the closest points of the two boxes' edges
 * that support the contact (extreme along +n on A, -n on B).  All points carry the pair's depth. */
static int clip_plane3(const double (*in)[3], int n, const double pn[3], double off, double (*out)[3], int* band) {
  int m = 0;
  for (int i = 0; i < n; ++i) {
    const double* a = in[(i + n - 1) % n];
    const double* b = in[i];
    const double da = dot3(pn, a) - off, db = dot3(pn, b) - off;   /* <= 0 inside */
    if (fabs(db) < BAND) *band |= OR_BAND_CLIP;
    const int ia = da <= 0.0, ib = db <= 0.0;
    if (ib) {
      if (!ia) {
        const double t = da / (da - db);
        for (int k = 0; k < 3; ++k) out[m][k] = a[k] + t * (b[k] - a[k]);
        ++m;
      }
      memcpy(out[m++], b, sizeof(double) * 3);
    } else if (ia) {
      const double t = da / (da - db);
      for (int k = 0; k < 3; ++k) out[m][k] = a[k] + t * (b[k] - a[k]);
      ++m;
    }
  }
  return m;
}

static int manifold_refface_R(const double heA[3], const double xA[3], const double RA[9],
                              const double heB[3], const double xB[3], const double RB[9],
                              const double n[3], double depth, int axis, or_manifold* m) {
  double t1[3], t2[3];
  tangent_basis(n, t1, t2);
  memcpy(m->normal, n, sizeof(double) * 3);
  memcpy(m->t1, t1, sizeof(double) * 3);
  memcpy(m->t2, t2, sizeof(double) * 3);
  m->depth = depth;
  m->npts = 0;
  double A[3][3], B[3][3];
  for (int i = 0; i < 3; ++i) { col3(RA, i, A[i]); col3(RB, i, B[i]); }
  if (axis >= 6) {
    /* edge-edge: the support edges along +n (A) and -n (B) */
    const int i = (axis - 6) / 3, j = (axis - 6) % 3;
    double pa[3], pb[3];
    for (int k = 0; k < 3; ++k) { pa[k] = xA[k]; pb[k] = xB[k]; }
    for (int q = 0; q < 3; ++q) {
      if (q != i) {
        const double sg = dot3(n, A[q]) >= 0.0 ? 1.0 : -1.0;
        for (int k = 0; k < 3; ++k) pa[k] += sg * heA[q] * A[q][k];
      }
      if (q != j) {
        const double sg = dot3(n, B[q]) >= 0.0 ? -1.0 : 1.0;
        for (int k = 0; k < 3; ++k) pb[k] += sg * heB[q] * B[q][k];
      }
    }
    /* closest points of the segments pa + s A_i (|s| <= heA_i), pb + t B_j (|t| <= heB_j) */
    double r[3];
    for (int k = 0; k < 3; ++k) r[k] = pa[k] - pb[k];
    const double a11 = 1.0, a22 = 1.0, a12 = dot3(A[i], B[j]);
    const double b1 = -dot3(A[i], r), b2 = dot3(B[j], r);
    const double det = a11 * a22 - a12 * a12;
    double sa = det > 1e-12 ? (b1 * a22 + a12 * b2) / det : 0.0;
    if (sa > heA[i]) sa = heA[i];
    if (sa < -heA[i]) sa = -heA[i];
    /* t minimising |pa + sa A_i - pb - t B_j| for this sa, clamped, then sa again for that t */
    double tb = dot3(B[j], r) + a12 * sa;
    if (tb > heB[j]) tb = heB[j];
    if (tb < -heB[j]) tb = -heB[j];
    sa = -dot3(A[i], r) + a12 * tb;
    if (sa > heA[i]) sa = heA[i];
    if (sa < -heA[i]) sa = -heA[i];
    for (int k = 0; k < 3; ++k)
      m->point[0][k] = 0.5 * ((pa[k] + sa * A[i][k]) + (pb[k] + tb * B[j][k]));
    m->slot[0] = 0;
    m->npts = 1;
    return 1;
  }
  const int refA = axis < 3;
  const double(*Rf)[3] = refA ? A : B;
  const double(*In)[3] = refA ? B : A;
  const double* heR = refA ? heA : heB;
  const double* heI = refA ? heB : heA;
  const double* xR = refA ? xA : xB;
  const double* xI = refA ? xB : xA;
  const int fi = refA ? axis : axis - 3;
  double u[3];
  for (int k = 0; k < 3; ++k) u[k] = refA ? n[k] : -n[k];
  /* reference face: centre, its plane offset along u, side axes */
  double cr[3];
  const double su = dot3(u, Rf[fi]) >= 0.0 ? 1.0 : -1.0;
  for (int k = 0; k < 3; ++k) cr[k] = xR[k] + su * heR[fi] * Rf[fi][k];
  const int s1 = (fi + 1) % 3, s2 = (fi + 2) % 3;
  /* incident face: most opposed to u */
  int fk = 0;
  double best = -1.0;
  for (int k = 0; k < 3; ++k) {
    const double d = fabs(dot3(u, In[k]));
    if (d > best) { best = d; fk = k; }
  }
  for (int k = 0; k < 3; ++k)
    if (k != fk && best - fabs(dot3(u, In[k])) < 1e-9) m->band |= OR_BAND_CLIP;
  const double sf = dot3(u, In[fk]) >= 0.0 ? -1.0 : 1.0;   /* the face whose normal opposes u */
  const int g1 = (fk + 1) % 3, g2 = (fk + 2) % 3;
  double poly[16][3], tmp[16][3];
  static const double cs[4][2] = {{1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
  for (int c = 0; c < 4; ++c)
    for (int k = 0; k < 3; ++k)
      poly[c][k] = xI[k] + sf * heI[fk] * In[fk][k] + cs[c][0] * heI[g1] * In[g1][k] + cs[c][1] * heI[g2] * In[g2][k];
  int np = 4;
  const int sides[4] = {s1, s1, s2, s2};
  const double sgn[4] = {1.0, -1.0, 1.0, -1.0};
  for (int e = 0; e < 4 && np > 0; ++e) {
    double pn[3];
    for (int k = 0; k < 3; ++k) pn[k] = sgn[e] * Rf[sides[e]][k];
    const double off = dot3(pn, cr) + heR[sides[e]];
    np = clip_plane3((const double(*)[3])poly, np, pn, off, tmp, &m->band);
    memcpy(poly, tmp, sizeof(double) * 3 * (size_t)np);
  }
  /* the vertices on or below the reference face, lifted halfway to it */
  double pts[16][3];
  int nk = 0;
  const double h = dot3(u, cr);
  for (int i = 0; i < np; ++i) {
    const double sep = h - dot3(u, poly[i]);
    if (fabs(sep) < BAND) m->band |= OR_BAND_CLIP;
    if (sep < 0.0) continue;
    for (int k = 0; k < 3; ++k) pts[nk][k] = poly[i][k] + 0.5 * sep * u[k];
    ++nk;
  }
  if (nk == 0) {
    /* nothing below the reference face: the silhouettes' empty-clip point */
    m->band |= OR_BAND_EMPTY;
    return manifold_box_R(heA, xA, RA, heB, xB, RB, n, depth, m);
  }
  static const double diag[4][2] = {{1.0, 1.0}, {-1.0, 1.0}, {-1.0, -1.0}, {1.0, -1.0}};
  int chosen[4], nchosen = 0;
  for (int s = 0; s < 4; ++s) {
    int bi = 0;
    double bv = diag[s][0] * dot3(pts[0], t1) + diag[s][1] * dot3(pts[0], t2);
    for (int i = 1; i < nk; ++i) {
      const double val = diag[s][0] * dot3(pts[i], t1) + diag[s][1] * dot3(pts[i], t2);
      if (val > bv) { bv = val; bi = i; }
    }
    for (int i = 0; i < nk; ++i) {
      if (i == bi) continue;
      const double val = diag[s][0] * dot3(pts[i], t1) + diag[s][1] * dot3(pts[i], t2);
      if (bv - val < BAND) m->band |= OR_BAND_CLIP;
    }
    int dup = 0;
    for (int c = 0; c < nchosen; ++c) dup |= (chosen[c] == bi);
    if (dup) continue;
    chosen[nchosen++] = bi;
    const int j = m->npts++;
    memcpy(m->point[j], pts[bi], sizeof(double) * 3);
    m->slot[j] = s;
  }
  return 1;
}

int or_manifold_refface(const double heA[3], const double xA[3], const double qA[4],
                        const double heB[3], const double xB[3], const double qB[4],
                        const double normal[3], double depth, int axis, or_manifold* out) {
  double RA[9], RB[9];
  or_quat_to_rot(qA, RA);
  or_quat_to_rot(qB, RB);
  memset(out, 0, sizeof(*out));
  out->b = 1;
  return manifold_refface_R(heA, xA, RA, heB, xB, RB, normal, depth, axis, out);
}

int or_manifold_box(const double heA[3], const double xA[3], const double qA[4],
                    const double heB[3], const double xB[3], const double qB[4],
                    const double normal[3], double depth, or_manifold* out) {
  double RA[9], RB[9];
  or_quat_to_rot(qA, RA);
  or_quat_to_rot(qB, RB);
  memset(out, 0, sizeof(*out));
  out->b = 1;
  return manifold_box_R(heA, xA, RA, heB, xB, RB, normal, depth, out);
}

static int manifold_ground_R(const double he[3], const double x[3], const double R[9], or_manifold* m) {
  double c[8][3];
  int below[8], nbelow = 0;
  for (int k = 0; k < 8; ++k) {
    box_corner(he, x, R, k, c[k]);
    if (fabs(c[k][2]) < BAND) m->band |= OR_BAND_GROUND;
    if (c[k][2] < 0.0) below[nbelow++] = k;
  }
  if (nbelow == 0) return 0;
  /* keep the 4 deepest (ties: lower vertex index), then order by vertex index */
  int keep[8];
  int nk = nbelow;
  for (int i = 0; i < nbelow; ++i) keep[i] = below[i];
  if (nbelow > 4) {
    /* stable selection sort by depth */
    for (int i = 0; i < nbelow; ++i)
      for (int j = i + 1; j < nbelow; ++j)
        if (c[keep[j]][2] < c[keep[i]][2]) { int t = keep[i]; keep[i] = keep[j]; keep[j] = t; }
    if (c[keep[4]][2] - c[keep[3]][2] < BAND) m->band |= OR_BAND_GROUND;
    nk = 4;
    for (int i = 0; i < 4; ++i)
      for (int j = i + 1; j < 4; ++j)
        if (keep[j] < keep[i]) { int t = keep[i]; keep[i] = keep[j]; keep[j] = t; }
  }
  double n[3] = {0.0, 0.0, -1.0};
  double t1[3], t2[3];
  tangent_basis(n, t1, t2);
  memcpy(m->normal, n, sizeof(double) * 3);
  memcpy(m->t1, t1, sizeof(double) * 3);
  memcpy(m->t2, t2, sizeof(double) * 3);
  m->npts = nk;
  m->depth = 0.0;
  for (int i = 0; i < nk; ++i) {
    const double* p = c[keep[i]];
    m->point[i][0] = p[0];
    m->point[i][1] = p[1];
    m->point[i][2] = 0.5 * p[2];
    m->slot[i] = keep[i];
    if (-p[2] > m->depth) m->depth = -p[2];
  }
  return 1;
}

int or_manifold_ground(const double he[3], const double x[3], const double q[4], or_manifold* out) {
  double R[9];
  or_quat_to_rot(q, R);
  memset(out, 0, sizeof(*out));
  out->b = -1;
  out->axis = -1;
  return manifold_ground_R(he, x, R, out);
}

/* ------------------------------------------------------------------------------------------ */
/* PGS (Sec. "Contact Solver --- Projected Gauss-Seidel")                                     */
/* ------------------------------------------------------------------------------------------ */

/* relative velocity of B with respect to A at the contact, along d */
static double rel_vel(const double* vA, const double* wA, const double* vB, const double* wB,
                      const double rA[3], const double rB[3], const double d[3]) {
  double za[3] = {0, 0, 0}, zb[3] = {0, 0, 0};
  double ua[3], ub[3], a[3], b[3];
  if (!vA) { vA = za; wA = za; }
  if (!vB) { vB = zb; wB = zb; }
  cross3(wA, rA, ua);
  cross3(wB, rB, ub);
  for (int k = 0; k < 3; ++k) { a[k] = vA[k] + ua[k]; b[k] = vB[k] + ub[k]; }
  double r[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  return dot3(r, d);
}

/* Eq. (keff) along direction d */
static double eff_inv_mass(double invmA, const double* IA, double invmB, const double* IB,
                           const double rA[3], const double rB[3], const double d[3]) {
  double k = invmA + invmB;
  double c[3], ic[3], t[3];
  if (IA) {
    cross3(rA, d, c); mat_vec(IA, c, ic); cross3(ic, rA, t);
    k += dot3(d, t);
  }
  if (IB) {
    cross3(rB, d, c); mat_vec(IB, c, ic); cross3(ic, rB, t);
    k += dot3(d, t);
  }
  return k;
}

/* the coupling of two rows d1, d2 of one point: the off-diagonal entry J1 M^-1 J2^T of the
 * contact's inverse effective mass matrix, (m_A^-1 + m_B^-1) d1.d2 + sum (r x d1).I^-1 (r x d2) */
static double eff_inv_mass_cross(double invmA, const double* IA, double invmB, const double* IB,
                                 const double rA[3], const double rB[3], const double d1[3], const double d2[3]) {
  double k = (invmA + invmB) * dot3(d1, d2);
  double c1[3], c2[3], ic[3];
  if (IA) {
    cross3(rA, d1, c1); cross3(rA, d2, c2); mat_vec(IA, c2, ic);
    k += dot3(c1, ic);
  }
  if (IB) {
    cross3(rB, d1, c1); cross3(rB, d2, c2); mat_vec(IB, c2, ic);
    k += dot3(c1, ic);
  }
  return k;
}

/* the larger eigenvalue of the tangent block [[k1, k12], [k12, k2]] of a point: the step 1 / kt
 * along the slip never overshoots in any direction of the pair */
static double tangent_block_max(double k1, double k2, double k12) {
  const double h = 0.5 * (k1 - k2);
  return 0.5 * (k1 + k2) + sqrt(h * h + k12 * k12);
}

/* apply impulse P (along d, magnitude dl): A gets -P, B gets +P */
static void apply_impulse(double invmA, const double* IA, double* vA, double* wA,
                          double invmB, const double* IB, double* vB, double* wB,
                          const double rA[3], const double rB[3], const double d[3], double dl) {
  double P[3] = {dl * d[0], dl * d[1], dl * d[2]};
  double c[3], ic[3];
  if (vA) {
    cross3(rA, P, c); mat_vec(IA, c, ic);
    for (int k = 0; k < 3; ++k) { vA[k] -= invmA * P[k]; wA[k] -= ic[k]; }
  }
  if (vB) {
    cross3(rB, P, c); mat_vec(IB, c, ic);
    for (int k = 0; k < 3; ++k) { vB[k] += invmB * P[k]; wB[k] += ic[k]; }
  }
}

typedef struct {
  const double* invm;
  const double* Iinv;   /* [nb][9] */
  const double* x;
  double* v;
  double* w;
  const uint8_t* dyn;   /* 1 = dynamic (written by the solver) */
} body_view;

static void contact_refs(const body_view* bv, const or_manifold* m,
                         double* invmA, const double** IA, double** vA, double** wA,
                         double* invmB, const double** IB, double** vB, double** wB) {
  *invmA = 0.0; *IA = NULL; *vA = NULL; *wA = NULL;
  *invmB = 0.0; *IB = NULL; *vB = NULL; *wB = NULL;
  if (bv->dyn[m->a]) {
    *invmA = bv->invm[m->a]; *IA = bv->Iinv + 9 * m->a; *vA = bv->v + 3 * m->a; *wA = bv->w + 3 * m->a;
  }
  if (m->b >= 0 && bv->dyn[m->b]) {
    *invmB = bv->invm[m->b]; *IB = bv->Iinv + 9 * m->b; *vB = bv->v + 3 * m->b; *wB = bv->w + 3 * m->b;
  }
}

static void lever_arms(const body_view* bv, const or_manifold* m, int i, double rA[3], double rB[3]) {
  for (int k = 0; k < 3; ++k) {
    rA[k] = m->point[i][k] - bv->x[3 * m->a + k];
    rB[k] = (m->b >= 0) ? m->point[i][k] - bv->x[3 * m->b + k] : 0.0;
  }
}

static void prep_k(const body_view* bv, or_manifold* ms, int nm) {
  for (int c = 0; c < nm; ++c) {
    or_manifold* m = &ms[c];
    double invmA, invmB; const double *IA, *IB; double *vA, *wA, *vB, *wB;
    contact_refs(bv, m, &invmA, &IA, &vA, &wA, &invmB, &IB, &vB, &wB);
    for (int i = 0; i < m->npts; ++i) {
      double rA[3], rB[3];
      lever_arms(bv, m, i, rA, rB);
      m->k[i][0] = eff_inv_mass(invmA, IA, invmB, IB, rA, rB, m->normal);
      m->k[i][1] = eff_inv_mass(invmA, IA, invmB, IB, rA, rB, m->t1);
      m->k[i][2] = eff_inv_mass(invmA, IA, invmB, IB, rA, rB, m->t2);
      m->k12[i] = eff_inv_mass_cross(invmA, IA, invmB, IB, rA, rB, m->t1, m->t2);
    }
  }
}

/* pre-solve restitution targets: -e v_n- for a point approaching faster than vth (v_n- < -vth, its
 * normal velocity before any impulse of the step), else 0 (only with the bias option) */
static void prep_bias(const body_view* bv, or_manifold* ms, int nm, double e, double vth) {
  for (int c = 0; c < nm; ++c) {
    or_manifold* m = &ms[c];
    double invmA, invmB; const double *IA, *IB; double *vA, *wA, *vB, *wB;
    contact_refs(bv, m, &invmA, &IA, &vA, &wA, &invmB, &IB, &vB, &wB);
    for (int i = 0; i < m->npts; ++i) {
      double rA[3], rB[3];
      lever_arms(bv, m, i, rA, rB);
      const double vn = rel_vel(vA, wA, vB, wB, rA, rB, m->normal);
      m->vbias[i] = vn < -vth ? -e * vn : 0.0;
    }
  }
}

/* friction and restitution options of a solve */
typedef struct {
  double mu, e;
  int cone;      /* 0: each tangent clipped to +-mu lambda_n (Eq. (coulomb_pgs)); 1: the tangent pair
                    projected onto the disc of radius mu lambda_n (the cone of the PGS figure) */
  int bias;      /* 0: (1 + e) times the current normal velocity every iteration (Eq. (lambda_n) as
                    printed); 1: a pre-solve target -e min(0, v_n-) per point (m->vbias) */
} solve_opts;

/* the tangent pair (l1, l2) projected onto the disc of radius b */
static void disc_project(double* l1, double* l2, double b) {
  const double s = sqrt(*l1 * *l1 + *l2 * *l2);
  if (s > b) {
    const double f = s > 0.0 ? b / s : 0.0;
    *l1 *= f;
    *l2 *= f;
  }
}

/* one Gauss-Seidel pass over the manifolds in array order */
static void pgs_sweep(const body_view* bv, or_manifold* ms, int nm, const solve_opts* o) {
  const double mu = o->mu, e = o->e;
  for (int c = 0; c < nm; ++c) {
    or_manifold* m = &ms[c];
    double invmA, invmB; const double *IA, *IB; double *vA, *wA, *vB, *wB;
    contact_refs(bv, m, &invmA, &IA, &vA, &wA, &invmB, &IB, &vB, &wB);
    for (int i = 0; i < m->npts; ++i) {
      double rA[3], rB[3];
      lever_arms(bv, m, i, rA, rB);
      /* Eq. (lambda_n): normal impulse with restitution, accumulated and clamped at 0 */
      double vn = rel_vel(vA, wA, vB, wB, rA, rB, m->normal);
      double dl = o->bias ? (m->vbias[i] - vn) / m->k[i][0] : -(1.0 + e) * vn / m->k[i][0];
      double ln = m->lam[i][0] + dl;
      if (ln < 0.0) ln = 0.0;
      apply_impulse(invmA, IA, vA, wA, invmB, IB, vB, wB, rA, rB, m->normal, ln - m->lam[i][0]);
      m->lam[i][0] = ln;
      double bound = mu * m->lam[i][0];
      if (o->cone) {
        /* both tangent rows from the same velocities, with one inverse effective mass (the larger
         * eigenvalue of the pair's 2 x 2 block) so that the update points against the slip
         * velocity and overshoots in no direction; the pair is then projected onto the disc */
        const double kt = tangent_block_max(m->k[i][1], m->k[i][2], m->k12[i]);
        double v1 = rel_vel(vA, wA, vB, wB, rA, rB, m->t1);
        double v2 = rel_vel(vA, wA, vB, wB, rA, rB, m->t2);
        double l1 = m->lam[i][1] - v1 / kt;
        double l2 = m->lam[i][2] - v2 / kt;
        disc_project(&l1, &l2, bound);
        apply_impulse(invmA, IA, vA, wA, invmB, IB, vB, wB, rA, rB, m->t1, l1 - m->lam[i][1]);
        apply_impulse(invmA, IA, vA, wA, invmB, IB, vB, wB, rA, rB, m->t2, l2 - m->lam[i][2]);
        m->lam[i][1] = l1;
        m->lam[i][2] = l2;
        continue;
      }
      /* Eq. (coulomb_pgs): each tangent clipped to +-mu lambda_n */
      for (int t = 1; t <= 2; ++t) {
        const double* d = (t == 1) ? m->t1 : m->t2;
        double vt = rel_vel(vA, wA, vB, wB, rA, rB, d);
        double lt = m->lam[i][t] - vt / m->k[i][t];
        if (lt < -bound) lt = -bound;
        if (lt > bound) lt = bound;
        apply_impulse(invmA, IA, vA, wA, invmB, IB, vB, wB, rA, rB, d, lt - m->lam[i][t]);
        m->lam[i][t] = lt;
      }
    }
  }
}

/* natural-map residual of every row at the current velocities: normal min(k lambda, w - target);
 * tangents k (lambda - P(lambda - w / k)) with P the solver's clip (box) or disc projection */
static void residual(const body_view* bv, const or_manifold* ms, int nm, const solve_opts* o, double res[2]) {
  const double mu = o->mu;
  double sum = 0.0, mx = 0.0;
  long rows = 0;
  for (int c = 0; c < nm; ++c) {
    const or_manifold* m = &ms[c];
    double invmA, invmB; const double *IA, *IB; double *vA, *wA, *vB, *wB;
    contact_refs(bv, m, &invmA, &IA, &vA, &wA, &invmB, &IB, &vB, &wB);
    for (int i = 0; i < m->npts; ++i) {
      double rA[3], rB[3];
      lever_arms(bv, m, i, rA, rB);
      double wn = rel_vel(vA, wA, vB, wB, rA, rB, m->normal) - (o->bias ? m->vbias[i] : 0.0);
      double kl = m->k[i][0] * m->lam[i][0];
      double r = kl < wn ? kl : wn;
      sum += r * r; if (fabs(r) > mx) mx = fabs(r);
      double bound = mu * m->lam[i][0];
      double cl[3], kr[3];
      const double kt = tangent_block_max(m->k[i][1], m->k[i][2], m->k12[i]);
      for (int t = 1; t <= 2; ++t) {
        const double* d = (t == 1) ? m->t1 : m->t2;
        double wt = rel_vel(vA, wA, vB, wB, rA, rB, d);
        kr[t] = o->cone ? kt : m->k[i][t];
        cl[t] = m->lam[i][t] - wt / kr[t];
        if (!o->cone) {
          if (cl[t] < -bound) cl[t] = -bound;
          if (cl[t] > bound) cl[t] = bound;
        }
      }
      if (o->cone) disc_project(&cl[1], &cl[2], bound);
      for (int t = 1; t <= 2; ++t) {
        double rt = kr[t] * (m->lam[i][t] - cl[t]);
        sum += rt * rt; if (fabs(rt) > mx) mx = fabs(rt);
      }
      rows += 3;
    }
  }
  res[0] = rows ? sqrt(sum / (double)rows) : 0.0;
  res[1] = mx;
}

void or_pgs(int nb, const double* invm, const double* Iinv, const double* x, double* v, double* w,
            int nm, or_manifold* m, double mu, double restitution, int iters, double res[2]) {
  or_pgs_ex(nb, invm, Iinv, x, v, w, nm, m, mu, restitution, 0, 0, iters, res);
}

void or_pgs_ex(int nb, const double* invm, const double* Iinv, const double* x, double* v, double* w,
               int nm, or_manifold* m, double mu, double restitution, int cone, int bias, int iters,
               double res[2]) {
  uint8_t* dyn = (uint8_t*)malloc((size_t)(nb > 0 ? nb : 1));
  for (int i = 0; i < nb; ++i) dyn[i] = invm[i] > 0.0;
  body_view bv = {invm, Iinv, x, v, w, dyn};
  const solve_opts o = {mu, restitution, cone, bias};
  prep_k(&bv, m, nm);
  if (bias) prep_bias(&bv, m, nm, restitution, 0.0);
  for (int it = 0; it < iters; ++it) pgs_sweep(&bv, m, nm, &o);
  residual(&bv, m, nm, &o, res);
  free(dyn);
}

/* ------------------------------------------------------------------------------------------ */
/* broadphase (Eq. (aabb))                                                                     */
/* ------------------------------------------------------------------------------------------ */

static void aabb_half(const double he[3], const double R[9], double h[3]) {
  for (int k = 0; k < 3; ++k) h[k] = fabs(R[3 * k]) * he[0] + fabs(R[3 * k + 1]) * he[1] + fabs(R[3 * k + 2]) * he[2];
}

static int broadphase_R(int nb, const double* x, const double* h, const uint8_t* act, const uint8_t* dyn,
                        double margin, int32_t* pairs, int cap) {
  int n = 0;
  for (int i = 0; i < nb; ++i) {
    if (!act[i]) continue;
    for (int j = i + 1; j < nb; ++j) {
      if (!act[j] || (!dyn[i] && !dyn[j])) continue;
      int ov = 1;
      for (int k = 0; k < 3; ++k)
        if (!(fabs(x[3 * i + k] - x[3 * j + k]) <= h[3 * i + k] + h[3 * j + k] + margin)) ov = 0;
      if (ov) {
        if (n < cap) { pairs[2 * n] = i; pairs[2 * n + 1] = j; }
        ++n;
      }
    }
    if (dyn[i] && x[3 * i + 2] - h[3 * i + 2] <= margin) {
      if (n < cap) { pairs[2 * n] = i; pairs[2 * n + 1] = -1; }
      ++n;
    }
  }
  return n;
}

int or_broadphase(int nb, const double* he, const double* mass, const double* x, const double* q,
                  const uint8_t* active, double margin, int32_t* pairs, int cap) {
  double* h = (double*)malloc(sizeof(double) * 3 * (size_t)(nb > 0 ? nb : 1));
  uint8_t* dyn = (uint8_t*)malloc((size_t)(nb > 0 ? nb : 1));
  for (int i = 0; i < nb; ++i) {
    double R[9];
    or_quat_to_rot(q + 4 * i, R);
    aabb_half(he + 3 * i, R, h + 3 * i);
    dyn[i] = active[i] && mass[i] > 0.0;
  }
  int n = broadphase_R(nb, x, h, active, dyn, margin, pairs, cap);
  free(h);
  free(dyn);
  return n;
}

/* ------------------------------------------------------------------------------------------ */
/* learned warm start: features and the per-contact MLP                                        */
/* ------------------------------------------------------------------------------------------ */

double or_bf16(double x) {
  /* to single precision, then to bfloat16 with round-to-nearest-even on the float's bits */
  float f = (float)x;
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (double)f;   /* inf / nan unchanged */
  u += 0x7fffu + ((u >> 16) & 1u);
  u &= 0xffff0000u;
  memcpy(&f, &u, 4);
  return (double)f;
}

static double gelu(double x) { return 0.5 * x * (1.0 + erf(x / sqrt(2.0))); }

void or_mlp_forward(const double* mlp, const double f[OR_NFEAT], double y[3]) {
  const double* W1 = mlp;
  const double* b1 = W1 + OR_NFEAT * OR_HIDDEN;
  const double* W2 = b1 + OR_HIDDEN;
  const double* b2 = W2 + OR_HIDDEN * OR_HIDDEN;
  const double* W3 = b2 + OR_HIDDEN;
  const double* b3 = W3 + OR_HIDDEN * 3;
  const double* mean = b3 + 3;
  const double* sd = mean + OR_NFEAT;
  double x0[OR_NFEAT], h1[OR_HIDDEN], h2[OR_HIDDEN];
  for (int i = 0; i < OR_NFEAT; ++i) x0[i] = or_bf16((f[i] - mean[i]) / sd[i]);
  for (int j = 0; j < OR_HIDDEN; ++j) {
    double s = b1[j];
    for (int i = 0; i < OR_NFEAT; ++i) s += x0[i] * W1[i * OR_HIDDEN + j];
    h1[j] = or_bf16(gelu(s));
  }
  for (int j = 0; j < OR_HIDDEN; ++j) {
    double s = b2[j];
    for (int i = 0; i < OR_HIDDEN; ++i) s += h1[i] * W2[i * OR_HIDDEN + j];
    h2[j] = or_bf16(gelu(s));
  }
  for (int j = 0; j < 3; ++j) {
    double s = b3[j];
    for (int i = 0; i < OR_HIDDEN; ++i) s += h2[i] * W3[i * 3 + j];
    y[j] = s;
  }
}

/* the 24 features of point i of manifold m, at the pre-solve velocities:
 * contact-frame x_B - x_A (3), q_A^-1 q_B with w >= 0 (4), world normal (3), depth (1), mu (1),
 * previous-step impulses of the same key in the outputs' units, lambda_d k_d / (|g| dt) with
 * this step's k (3, zero if new), contact-frame r_A and r_B (6), contact-frame relative velocity
 * of the contact point (3).  The ground stands in as a body at (x_A, y_A, 0) with the identity
 * orientation.  m->k must hold this step's inverse effective masses. */
static void point_features(const or_manifold* m, int i, const double* x, const double* q, const double* v,
                           const double* w, const uint8_t* dyn, double mu, const double prev_lam[3],
                           double gdt, double f[OR_NFEAT]) {
  const double* F[3] = {m->normal, m->t1, m->t2};
  const double* xa = x + 3 * m->a;
  double xb[3] = {xa[0], xa[1], 0.0};
  double qb[4] = {1.0, 0.0, 0.0, 0.0};
  if (m->b >= 0) {
    for (int k = 0; k < 3; ++k) xb[k] = x[3 * m->b + k];
    for (int k = 0; k < 4; ++k) qb[k] = q[4 * m->b + k];
  }
  const double* qa = q + 4 * m->a;
  double d[3] = {xb[0] - xa[0], xb[1] - xa[1], xb[2] - xa[2]};
  int o = 0;
  for (int k = 0; k < 3; ++k) f[o++] = dot3(F[k], d);
  /* conj(qa) (x) qb */
  double aw = qa[0], ax = -qa[1], ay = -qa[2], az = -qa[3];
  double bw = qb[0], bx = qb[1], by = qb[2], bz = qb[3];
  double r[4] = {aw * bw - ax * bx - ay * by - az * bz, aw * bx + ax * bw + ay * bz - az * by,
                 aw * by - ax * bz + ay * bw + az * bx, aw * bz + ax * by - ay * bx + az * bw};
  double sg = r[0] < 0.0 ? -1.0 : 1.0;
  for (int k = 0; k < 4; ++k) f[o++] = sg * r[k];
  for (int k = 0; k < 3; ++k) f[o++] = m->normal[k];
  f[o++] = m->depth;
  f[o++] = mu;
  for (int k = 0; k < 3; ++k) f[o++] = prev_lam[k] * m->k[i][k] / gdt;
  double rA[3], rB[3];
  for (int k = 0; k < 3; ++k) {
    rA[k] = m->point[i][k] - xa[k];
    rB[k] = m->point[i][k] - xb[k];
  }
  for (int k = 0; k < 3; ++k) f[o++] = dot3(F[k], rA);
  for (int k = 0; k < 3; ++k) f[o++] = dot3(F[k], rB);
  const double z[3] = {0.0, 0.0, 0.0};
  const double* vA = dyn[m->a] ? v + 3 * m->a : z;
  const double* wA = dyn[m->a] ? w + 3 * m->a : z;
  const double* vB = (m->b >= 0 && dyn[m->b]) ? v + 3 * m->b : z;
  const double* wB = (m->b >= 0 && dyn[m->b]) ? w + 3 * m->b : z;
  double ua[3], ub[3], rel[3];
  cross3(wA, rA, ua);
  cross3(wB, rB, ub);
  for (int k = 0; k < 3; ++k) rel[k] = (vB[k] + ub[k]) - (vA[k] + ua[k]);
  for (int k = 0; k < 3; ++k) f[o++] = dot3(F[k], rel);
}

/* ------------------------------------------------------------------------------------------ */
/* one tower step                                                                              */
/* ------------------------------------------------------------------------------------------ */

static void quat_normalise(double q[4]) {
  double l = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; ++k) q[k] /= l;
}

static int find_prev(const or_manifold* prev, int nprev, const or_manifold* m, int slot, double lam[3]) {
  for (int c = 0; c < nprev; ++c) {
    const or_manifold* p = &prev[c];
    if (p->a != m->a || p->b != m->b) continue;
    if (dot3(p->normal, m->normal) <= 0.95) return 0;
    for (int i = 0; i < p->npts; ++i)
      if (p->slot[i] == slot) { lam[0] = p->lam[i][0]; lam[1] = p->lam[i][1]; lam[2] = p->lam[i][2]; return 1; }
    return 0;
  }
  return 0;
}

static int substep(const or_params* P, double dt, int nb, const double* he, const double* mass,
                   double* x, double* q, double* v, double* w, uint8_t* active, double mu,
                   int npush, const or_push* push, int64_t step,
                   const or_manifold* prev, int nprev, or_manifold** ms_out, int* nm_out, or_stats* st,
                   double* feat_out, int feat_cap, int* nfeat_out) {
  const size_t NB = (size_t)(nb > 0 ? nb : 1);
  double* R = (double*)malloc(sizeof(double) * 9 * NB);
  double* Iinv = (double*)malloc(sizeof(double) * 9 * NB);
  double* Ib = (double*)malloc(sizeof(double) * 3 * NB);
  double* invm = (double*)malloc(sizeof(double) * NB);
  double* h = (double*)malloc(sizeof(double) * 3 * NB);
  uint8_t* dyn = (uint8_t*)malloc(NB);

  /* 1. external forces (gravity, pushes) for active dynamic bodies */
  for (int i = 0; i < nb; ++i) {
    dyn[i] = active[i] && mass[i] > 0.0;
    if (!dyn[i]) continue;
    for (int k = 0; k < 3; ++k) v[3 * i + k] += dt * P->gravity[k];
  }
  for (int r = 0; r < npush; ++r) {
    const or_push* pr = &push[r];
    if (step < pr->start || step >= (int64_t)pr->start + pr->steps) continue;
    int b = pr->body;
    if (b < 0 || b >= nb || !dyn[b]) continue;
    for (int k = 0; k < 3; ++k) v[3 * b + k] += dt * pr->force[k] / mass[b];
  }
  /* 2. frames */
  for (int i = 0; i < nb; ++i) {
    or_quat_to_rot(q + 4 * i, R + 9 * i);
    aabb_half(he + 3 * i, R + 9 * i, h + 3 * i);
    if (dyn[i]) {
      double I[3], d[3];
      or_box_inertia(mass[i], he + 3 * i, I);
      for (int k = 0; k < 3; ++k) { Ib[3 * i + k] = I[k]; d[k] = 1.0 / I[k]; }
      invm[i] = 1.0 / mass[i];
      rot_diag_rotT(R + 9 * i, d, Iinv + 9 * i);
    } else {
      invm[i] = 0.0;
      for (int k = 0; k < 9; ++k) Iinv[9 * i + k] = 0.0;
      for (int k = 0; k < 3; ++k) Ib[3 * i + k] = 0.0;
    }
  }
  /* 3. broadphase */
  /* room for 16 candidates per body; a denser scene is walked again with room for all */
  int cap = 16 * nb + 64;
  int32_t* pairs = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)cap);
  int ncand = broadphase_R(nb, x, h, active, dyn, P->margin, pairs, cap);
  if (ncand > cap) {
    free(pairs);
    cap = ncand;
    pairs = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)cap);
    ncand = broadphase_R(nb, x, h, active, dyn, P->margin, pairs, cap);
  }
  st->candidates += ncand;

  /* 4-5. narrowphase and manifolds, canonical (a, b) order with the ground last per body */
  or_manifold* ms = (or_manifold*)calloc((size_t)(ncand > 0 ? ncand : 1), sizeof(or_manifold));
  int nm = 0;
  for (int c = 0; c < ncand; ++c) {
    int a = pairs[2 * c], b = pairs[2 * c + 1];
    or_manifold* m = &ms[nm];
    memset(m, 0, sizeof(*m));
    m->a = a; m->b = b;
    if (b >= 0) {
      or_sat_result sr;
      sat_R(he + 3 * a, x + 3 * a, R + 9 * a, he + 3 * b, x + 3 * b, R + 9 * b, P->manifold_mode != 0, &sr);
      if (!sr.collide) continue;
      m->axis = sr.axis;
      m->band = sr.band;
      m->sigma = sr.sigma;
      if (P->manifold_mode)
        manifold_refface_R(he + 3 * a, x + 3 * a, R + 9 * a, he + 3 * b, x + 3 * b, R + 9 * b, sr.normal, sr.depth,
                           sr.axis, m);
      else
        manifold_box_R(he + 3 * a, x + 3 * a, R + 9 * a, he + 3 * b, x + 3 * b, R + 9 * b, sr.normal, sr.depth, m);
    } else {
      m->axis = -1;
      if (!manifold_ground_R(he + 3 * a, x + 3 * a, R + 9 * a, m)) continue;
      m->sigma = -m->depth;
    }
    ++nm;
  }
  st->manifolds += nm;

  /* 6. greedy first-fit colouring; conflicts only through dynamic bodies.  A tower below
   * mega_bodies takes its manifolds in canonical order.  A larger one is cut into partitions of
   * colour_partition bodies (by tower-local index) and takes them in four passes, each in
   * canonical order: (1) pairs inside a partition or with the ground; (2) pairs between
   * partitions p and p + 1 for even p; (3) the same for odd p; (4) pairs between partitions
   * further apart.  Within a pass, different partitions (or partition pairs) share no body. */
  uint64_t* used = (uint64_t*)calloc(NB, sizeof(uint64_t));
  int ncol = 0;
  const int parted = P->mega_bodies > 0 && nb >= P->mega_bodies;
  const int S = P->colour_partition > 0 ? P->colour_partition : 1024;
  for (int c = 0; c < nm; ++c) ms[c].colour = -1;
  for (int pass = 0; pass < (parted ? 4 : 1); ++pass) {
    for (int c = 0; c < nm; ++c) {
      or_manifold* m = &ms[c];
      if (parted) {
        const int pa = m->a / S, pb = m->b < 0 ? pa : m->b / S;
        const int want = pb == pa ? 0 : (pb == pa + 1 ? 1 + (pa & 1) : 3);
        if (want != pass) continue;
      }
      uint64_t u = 0;
      if (dyn[m->a]) u |= used[m->a];
      if (m->b >= 0 && dyn[m->b]) u |= used[m->b];
      int col = 0;
      while (col < MAX_COLOURS && (u >> col) & 1ull) ++col;
      if (col >= MAX_COLOURS) { st->error |= 1; continue; }   /* dropped */
      m->colour = col;
      if (dyn[m->a]) used[m->a] |= 1ull << col;
      if (m->b >= 0 && dyn[m->b]) used[m->b] |= 1ull << col;
      if (col + 1 > ncol) ncol = col + 1;
    }
  }
  int kept = 0;
  for (int c = 0; c < nm; ++c) {
    if (ms[c].colour < 0) continue;
    if (kept != c) ms[kept] = ms[c];
    ++kept;
  }
  nm = kept;
  free(used);
  /* processing order: by colour, canonical order within a colour (stable) */
  or_manifold* ord = (or_manifold*)malloc(sizeof(or_manifold) * (size_t)(nm > 0 ? nm : 1));
  int no = 0;
  for (int col = 0; col < ncol; ++col)
    for (int c = 0; c < nm; ++c)
      if (ms[c].colour == col) ord[no++] = ms[c];
  free(ms);
  st->colours = ncol;

  /* 7. prep and warm start */
  body_view bv = {invm, Iinv, x, v, w, dyn};
  const solve_opts so = {mu, P->restitution, P->friction_cone, P->restitution_bias};
  prep_k(&bv, ord, nm);
  /* a resting contact approaches at about |g| dt per step: twice that is the bounce threshold */
  if (P->restitution_bias) prep_bias(&bv, ord, nm, P->restitution, 2.0 * norm3(P->gravity) * dt);
  long npts = 0;
  for (int c = 0; c < nm; ++c) npts += ord[c].npts;
  const int learned = P->warm_start == 2 && P->mlp != NULL;
  double* feats = NULL;
  const double gdt = norm3(P->gravity) * dt;
  if (learned || feat_out) {
    feats = (double*)malloc(sizeof(double) * OR_NFEAT * (size_t)(npts > 0 ? npts : 1));
    long o = 0;
    for (int c = 0; c < nm; ++c) {
      const or_manifold* m = &ord[c];
      for (int i = 0; i < m->npts; ++i, ++o) {
        double l[3] = {0.0, 0.0, 0.0};
        if (prev) find_prev(prev, nprev, m, m->slot[i], l);
        point_features(m, i, x, q, v, w, dyn, mu, l, gdt, feats + OR_NFEAT * o);
      }
    }
  }
  {
    long o = 0;
    for (int c = 0; c < nm; ++c) {
      or_manifold* m = &ord[c];
      for (int i = 0; i < m->npts; ++i, ++o) {
        m->lam[i][0] = m->lam[i][1] = m->lam[i][2] = 0.0;
        if (P->warm_start == 1 && prev) {
          double l[3];
          if (find_prev(prev, nprev, m, m->slot[i], l)) { m->lam[i][0] = l[0]; m->lam[i][1] = l[1]; m->lam[i][2] = l[2]; }
        } else if (learned) {
          /* the network predicts the change of the dimensionless impulses lambda k / (|g| dt)
           * from the previous step's (input features 12..14) */
          double y[3];
          const double* f = feats + OR_NFEAT * o;
          or_mlp_forward(P->mlp, f, y);
          for (int d = 0; d < 3; ++d) y[d] += f[12 + d];
          double ln = (y[0] > 0.0 ? y[0] : 0.0) * gdt / m->k[i][0];
          double b = mu * ln;
          double l1 = y[1] * gdt / m->k[i][1], l2 = y[2] * gdt / m->k[i][2];
          if (P->friction_cone) {
            disc_project(&l1, &l2, b);
          } else {
            if (l1 < -b) l1 = -b;
            if (l1 > b) l1 = b;
            if (l2 < -b) l2 = -b;
            if (l2 > b) l2 = b;
          }
          m->lam[i][0] = ln; m->lam[i][1] = l1; m->lam[i][2] = l2;
        }
      }
    }
  }
  double* v_save = NULL;
  double* w_save = NULL;
  if (learned) {
    v_save = (double*)malloc(sizeof(double) * 3 * NB);
    w_save = (double*)malloc(sizeof(double) * 3 * NB);
    memcpy(v_save, v, sizeof(double) * 3 * (size_t)nb);
    memcpy(w_save, w, sizeof(double) * 3 * (size_t)nb);
  }
  if (P->warm_start == 1 || learned) {
    /* apply the initial impulses like solver impulses, in processing order */
    for (int c = 0; c < nm; ++c) {
      or_manifold* m = &ord[c];
      double invmA, invmB; const double *IA, *IB; double *vA, *wA, *vB, *wB;
      contact_refs(&bv, m, &invmA, &IA, &vA, &wA, &invmB, &IB, &vB, &wB);
      for (int i = 0; i < m->npts; ++i) {
        double rA[3], rB[3];
        lever_arms(&bv, m, i, rA, rB);
        apply_impulse(invmA, IA, vA, wA, invmB, IB, vB, wB, rA, rB, m->normal, m->lam[i][0]);
        apply_impulse(invmA, IA, vA, wA, invmB, IB, vB, wB, rA, rB, m->t1, m->lam[i][1]);
        apply_impulse(invmA, IA, vA, wA, invmB, IB, vB, wB, rA, rB, m->t2, m->lam[i][2]);
      }
    }
  }
  st->points += npts;

  /* 8. PGS; 9. residual.  A learned start runs mlp_iters sweeps; if the residual is still above
   * fallback_tau the solve is redone plainly (pre-solve velocities, zero impulses, iters sweeps). */
  const int iters = learned ? P->mlp_iters : P->iters;
  for (int it = 0; it < iters; ++it) pgs_sweep(&bv, ord, nm, &so);
  st->contact_iters += npts * (int64_t)iters;
  double res[2];
  residual(&bv, ord, nm, &so, res);
  if (learned && res[0] > P->fallback_tau) {
    memcpy(v, v_save, sizeof(double) * 3 * (size_t)nb);
    memcpy(w, w_save, sizeof(double) * 3 * (size_t)nb);
    for (int c = 0; c < nm; ++c)
      for (int i = 0; i < ord[c].npts; ++i) ord[c].lam[i][0] = ord[c].lam[i][1] = ord[c].lam[i][2] = 0.0;
    for (int it = 0; it < P->iters; ++it) pgs_sweep(&bv, ord, nm, &so);
    st->contact_iters += npts * (int64_t)P->iters;
    st->fallbacks += 1;
    residual(&bv, ord, nm, &so, res);
  }
  free(v_save);
  free(w_save);
  st->res_rms = res[0];
  st->res_max = res[1];
  if (feat_out) {
    long o = 0;
    for (int c = 0; c < nm; ++c) {
      const or_manifold* m = &ord[c];
      for (int i = 0; i < m->npts; ++i, ++o) {
        if (o >= feat_cap) continue;
        double* r = feat_out + (size_t)OR_FEAT_RECORD * o;
        memcpy(r, feats + OR_NFEAT * o, sizeof(double) * OR_NFEAT);
        for (int k = 0; k < 3; ++k) { r[OR_NFEAT + k] = m->k[i][k]; r[OR_NFEAT + 3 + k] = m->lam[i][k]; }
      }
    }
    *nfeat_out = (int)(npts < feat_cap ? npts : feat_cap);
  }
  free(feats);

  /* 10. integrate: x += dt v; q' = normalise(q + dt/2 [0,w] (x) q); keep L = I_w w */
  for (int i = 0; i < nb; ++i) {
    if (!dyn[i]) continue;
    double* xi = x + 3 * i; double* qi = q + 4 * i; double* vi = v + 3 * i; double* wi = w + 3 * i;
    for (int k = 0; k < 3; ++k) xi[k] += dt * vi[k];
    double Iw[9], L[3];
    rot_diag_rotT(R + 9 * i, Ib + 3 * i, Iw);
    mat_vec(Iw, wi, L);
    /* [0, w] (x) q, Hamilton product */
    double qw = qi[0], qx = qi[1], qy = qi[2], qz = qi[3];
    double dq[4];
    dq[0] = -(wi[0] * qx + wi[1] * qy + wi[2] * qz);
    dq[1] = wi[0] * qw + (wi[1] * qz - wi[2] * qy);
    dq[2] = wi[1] * qw + (wi[2] * qx - wi[0] * qz);
    dq[3] = wi[2] * qw + (wi[0] * qy - wi[1] * qx);
    for (int k = 0; k < 4; ++k) qi[k] += 0.5 * dt * dq[k];
    quat_normalise(qi);
    double R2[9], Iinv2[9], d[3];
    or_quat_to_rot(qi, R2);
    for (int k = 0; k < 3; ++k) d[k] = 1.0 / Ib[3 * i + k];
    rot_diag_rotT(R2, d, Iinv2);
    mat_vec(Iinv2, L, wi);
  }
  /* 11. Baumgarte position correction, per pair, canonical order */
  int* canon = (int*)malloc(sizeof(int) * (size_t)(nm > 0 ? nm : 1));
  for (int c = 0; c < nm; ++c) canon[c] = c;
  for (int i = 0; i < nm; ++i)       /* insertion sort by (a, b), ground last */
    for (int j = i; j > 0; --j) {
      const or_manifold* p = &ord[canon[j - 1]];
      const or_manifold* r = &ord[canon[j]];
      long kp = (long)p->a * 1000000L + (p->b < 0 ? 999999L : p->b);
      long kr = (long)r->a * 1000000L + (r->b < 0 ? 999999L : r->b);
      if (kp > kr) { int t = canon[j]; canon[j] = canon[j - 1]; canon[j - 1] = t; } else break;
    }
  for (int c = 0; c < nm; ++c) {
    const or_manifold* m = &ord[canon[c]];
    double ia = dyn[m->a] ? invm[m->a] : 0.0;
    double ib = (m->b >= 0 && dyn[m->b]) ? invm[m->b] : 0.0;
    if (ia + ib <= 0.0) continue;
    double corr = m->depth - P->slop;
    if (corr <= 0.0) continue;
    corr /= (ia + ib);
    for (int k = 0; k < 3; ++k) {
      if (ia > 0.0) x[3 * m->a + k] -= P->beta * ia * corr * m->normal[k];
      if (ib > 0.0) x[3 * m->b + k] += P->beta * ib * corr * m->normal[k];
    }
  }
  free(canon);

  *ms_out = ord;
  *nm_out = nm;
  free(pairs); free(R); free(Iinv); free(Ib); free(invm); free(h); free(dyn);
  return 0;
}

int or_step_tower(const or_params* p, int nb, const double* he, const double* mass,
                  double* x, double* q, double* v, double* w, uint8_t* active,
                  double mu, int npush, or_push* push, int64_t* step_counter, int n_steps,
                  const or_manifold* prev, int nprev,
                  or_manifold* mout, int mcap, int* nm_out, or_stats* st,
                  double* feat_out, int feat_cap, int* nfeat_out) {
  or_manifold* cur = NULL;
  int nfeat_dummy = 0;
  if (!nfeat_out) nfeat_out = &nfeat_dummy;
  *nfeat_out = 0;
  int ncur = 0;
  or_manifold* last = NULL;
  int nlast = 0;
  const int nsub = p->n_sub > 0 ? p->n_sub : 1;
  const double dt = p->dt / nsub;
  for (int s = 0; s < n_steps; ++s) {
    const int64_t step = *step_counter;
    for (int r = 0; r < npush; ++r)
      if (push[r].start == step && push[r].body >= 0 && push[r].body < nb)
        for (int k = 0; k < 3; ++k) push[r].x0[k] = x[3 * push[r].body + k];
    for (int sub = 0; sub < nsub; ++sub) {
      const or_manifold* pv = last ? last : prev;
      int npv = last ? nlast : nprev;
      const int final_sub = (s == n_steps - 1) && (sub == nsub - 1);
      substep(p, dt, nb, he, mass, x, q, v, w, active, mu, npush, push, step, pv, npv, &cur, &ncur, st,
              final_sub ? feat_out : NULL, feat_cap, nfeat_out);
      free(last);
      last = cur; nlast = ncur;
      cur = NULL;
    }
    /* withdrawal: a pushed body that moved far enough along its push leaves the tower */
    for (int r = 0; r < npush; ++r) {
      or_push* pr = &push[r];
      int b = pr->body;
      if (pr->withdraw <= 0.0 || step < pr->start || b < 0 || b >= nb || !active[b]) continue;
      double dx[3] = {x[3 * b] - pr->x0[0], x[3 * b + 1] - pr->x0[1], x[3 * b + 2] - pr->x0[2]};
      if (dot3(dx, pr->force) >= pr->withdraw * norm3(pr->force)) {
        active[b] = 0;
        for (int k = 0; k < 3; ++k) { v[3 * b + k] = 0.0; w[3 * b + k] = 0.0; }
      }
    }
    *step_counter += 1;
    st->steps += 1;
  }
  int n = nlast;
  if (mout) {
    if (n > mcap) { st->error |= 2; n = mcap; }
    if (n > 0) memcpy(mout, last, sizeof(or_manifold) * (size_t)n);
  }
  if (nm_out) *nm_out = nlast;
  free(last);
  return 0;
}
