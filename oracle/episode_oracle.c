/*
 * FP64 oracle of the episode criteria (Sec. "Stability Detection and Collapse").
 *
 * TEST INFRASTRUCTURE ONLY, like jenga_oracle.c: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.
 *
 *  - support polygon, Eq. (stability): the convex hull (Andrew's monotone chain, collinear points
 *    dropped) of the horizontal corners of every block whose lowest point is within eps of the
 *    ground; the margin is the smallest signed distance from the centre of mass to the hull's
 *    edge lines (positive inside);
 *  - composite collapse criterion, Eq. (collapse): displacement, kinetic energy and tilt;
 *  - simulate_until_rest (Sec. "Full Floor Contact Simulation"): after the collapse the tower
 *    runs until its kinetic energy drops below a threshold, or a fixed number of steps.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "jenga_oracle.h"

static const double kPi = 3.14159265358979323846;

typedef struct {
  double x, y;
} pt2;

static int cmp_pt(const void* a, const void* b) {
  const pt2* p = (const pt2*)a;
  const pt2* q = (const pt2*)b;
  if (p->x < q->x) return -1;
  if (p->x > q->x) return 1;
  if (p->y < q->y) return -1;
  if (p->y > q->y) return 1;
  return 0;
}

static double cross2(pt2 o, pt2 a, pt2 b) { return (a.x - o.x) * (b.y - o.y) - (a.y - o.y) * (b.x - o.x); }

/* Counter-clockwise hull of n points into h (capacity 2n); returns its vertex count.  Points on
 * an edge and duplicates are dropped. */
static int hull_ccw(pt2* p, int n, pt2* h) {
  if (n <= 0) return 0;
  qsort(p, (size_t)n, sizeof(pt2), cmp_pt);
  int k = 0;
  for (int i = 0; i < n; ++i) {
    while (k >= 2 && cross2(h[k - 2], h[k - 1], p[i]) <= 0.0) --k;
    h[k++] = p[i];
  }
  for (int i = n - 2, lo = k + 1; i >= 0; --i) {
    while (k >= lo && cross2(h[k - 2], h[k - 1], p[i]) <= 0.0) --k;
    h[k++] = p[i];
  }
  return k > 1 ? k - 1 : k;   /* the last point repeats the first */
}

void or_episode_eval(const or_episode_params* E, int nb, const double* he, const double* mass,
                        const double* x, const double* q, const double* v, const double* w,
                        const uint8_t* active, const double* x0, or_episode_metrics* out) {
  memset(out, 0, sizeof(*out));
  const double cos_th = cos(E->theta_deg * kPi / 180.0);
  double msum = 0.0, cx = 0.0, cy = 0.0, ek = 0.0, dx_max = 0.0, rzz_min = 1.0;
  int c_d = 0, nsup = 0;
  pt2* pts = (pt2*)malloc(sizeof(pt2) * (size_t)(8 * (nb > 0 ? nb : 1)));
  for (int i = 0; i < nb; ++i) {
    if (!active[i] || !(mass[i] > 0.0)) continue;
    const double m = mass[i];
    double R[9], I[3];
    or_quat_to_rot(q + 4 * i, R);
    or_box_inertia(m, he + 3 * i, I);
    /* kinetic energy: translation plus rotation with the body-frame inertia of Eq. (inertia) */
    const double* vi = v + 3 * i;
    const double* wi = w + 3 * i;
    double wb[3];
    for (int k = 0; k < 3; ++k) wb[k] = R[k] * wi[0] + R[3 + k] * wi[1] + R[6 + k] * wi[2];   /* R^T w */
    ek += 0.5 * m * (vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2]);
    ek += 0.5 * (I[0] * wb[0] * wb[0] + I[1] * wb[1] * wb[1] + I[2] * wb[2] * wb[2]);
    /* displacement from the episode's start, against half the block's own length */
    const double d[3] = {x[3 * i] - x0[3 * i], x[3 * i + 1] - x0[3 * i + 1], x[3 * i + 2] - x0[3 * i + 2]};
    const double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (dn > dx_max) dx_max = dn;
    if (dn > E->fd * 2.0 * he[3 * i]) c_d = 1;
    /* tilt: the angle between the block's thickness axis and the vertical */
    if (R[8] < rzz_min) rzz_min = R[8];
    /* centre of mass */
    msum += m;
    cx += m * x[3 * i];
    cy += m * x[3 * i + 1];
    /* a supporting block: its lowest point within eps of the ground; all 8 corners count */
    const double hz = fabs(R[6]) * he[3 * i] + fabs(R[7]) * he[3 * i + 1] + fabs(R[8]) * he[3 * i + 2];
    if (x[3 * i + 2] - hz <= E->eps) {
      for (int c = 0; c < 8; ++c) {
        const double s[3] = {(c & 1) ? he[3 * i] : -he[3 * i], (c & 2) ? he[3 * i + 1] : -he[3 * i + 1],
                             (c & 4) ? he[3 * i + 2] : -he[3 * i + 2]};
        pts[nsup].x = x[3 * i] + R[0] * s[0] + R[1] * s[1] + R[2] * s[2];
        pts[nsup].y = x[3 * i + 1] + R[3] * s[0] + R[4] * s[1] + R[5] * s[2];
        ++nsup;
      }
    }
  }
  out->ek = ek;
  out->dx_max = dx_max;
  out->theta_max = acos(rzz_min < -1.0 ? -1.0 : rzz_min);
  if (msum > 0.0) { out->com[0] = cx / msum; out->com[1] = cy / msum; }
  pt2* h = (pt2*)malloc(sizeof(pt2) * (size_t)(2 * (nsup > 0 ? nsup : 1)));
  const int nh = hull_ccw(pts, nsup, h);
  out->n_support = nh;
  double margin = -INFINITY;
  if (nh >= 3) {
    const pt2 c = {out->com[0], out->com[1]};
    margin = INFINITY;
    for (int k = 0; k < nh; ++k) {
      const pt2 a = h[k], b = h[(k + 1) % nh];
      const double len = sqrt((b.x - a.x) * (b.x - a.x) + (b.y - a.y) * (b.y - a.y));
      const double dist = cross2(a, b, c) / len;
      if (dist < margin) margin = dist;
    }
  }
  out->margin = margin;
  out->c_d = c_d;
  out->c_k = ek > E->ek_collapse;
  out->c_theta = rzz_min < cos_th;
  free(h);
  free(pts);
}

/* One step of a tower under the episode rules: a held tower (at rest after a collapse) does not
 * move; after the collapse no push acts and no pushed block is withdrawn any more.  The criteria
 * are evaluated on the state at the end of the step. */
int or_step_episode(const or_params* p, const or_episode_params* E, int nb, const double* he, const double* mass,
                    double* x, double* q, double* v, double* w, uint8_t* active, double mu, int npush,
                    or_push* push, int64_t* step_counter, const double* x0, or_episode_state* es,
                    const or_manifold* prev, int nprev, or_manifold* mout, int mcap, int* nm_out, or_stats* st) {
  const int64_t step = *step_counter;
  if (es->done) {
    *step_counter += 1;
    st->steps += 1;
    if (nm_out) *nm_out = 0;
    return 0;
  }
  if (es->collapsed) {
    for (int r = 0; r < npush; ++r) {
      const int64_t end = (int64_t)push[r].start + push[r].steps;
      if (end > (int64_t)es->collapse_step + 1) {
        const int64_t keep = (int64_t)es->collapse_step + 1 - push[r].start;
        push[r].steps = keep > 0 ? (int32_t)keep : 0;
      }
      push[r].withdraw = 0.0;
    }
  }
  or_step_tower(p, nb, he, mass, x, q, v, w, active, mu, npush, push, step_counter, 1, prev, nprev, mout, mcap,
                nm_out, st, NULL, 0, NULL);
  or_episode_eval(E, nb, he, mass, x, q, v, w, active, x0, &es->last);
  if (!es->collapsed) {
    if (es->last.c_d && es->last.c_k && es->last.c_theta) {
      es->collapsed = 1;
      es->collapse_step = (int32_t)step;
    } else {
      es->imbalance = -es->last.margin;
    }
  }
  if (es->collapsed) {
    if (es->last.ek < E->ek_rest) {
      es->done = 1;
      es->rest_step = (int32_t)step;
    } else if (step - es->collapse_step >= E->rest_steps) {
      es->done = 1;
      es->rest_step = -1;
    }
  }
  return 0;
}
