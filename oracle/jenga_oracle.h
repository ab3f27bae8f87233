/*
 * FP64 CPU oracle for batched stepping of towers of oriented boxes.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  The product path (the HIP
 * library) never links, includes or calls it, and shares no code with it.
 *
 * Everything is double precision and single threaded per tower.  A "tower" is an
 * independent world: bodies indexed 0..nb-1, plus a static ground half-space z <= 0.
 * Arrays are row-major: vec3 arrays are [nb][3], quaternions [nb][4] as [w,x,y,z].
 */
#ifndef JENGA_ORACLE_H
#define JENGA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double gravity[3];     /* m/s^2, (0,0,-9.81) (Sec. Equations of Motion) */
  double dt;             /* step length, 1/240 s */
  double restitution;    /* e in Eq. (lambda_n), 0.10 */
  double beta;           /* Baumgarte factor, Eq. (baumgarte), 0.35 */
  double slop;           /* Baumgarte slop, 0.4 mm */
  double margin;         /* AABB margin epsilon, Eq. (aabb), 2 mm */
  int32_t n_sub;         /* substeps per step (each runs the whole pipeline with dt/n_sub) */
  int32_t iters;         /* PGS iterations */
  int32_t warm_start;    /* 0: zero initial impulses, 1: previous step's impulses by key,
                            2: learned (MLP) initial impulses, plain solve as the fallback */
  int32_t mlp_iters;     /* PGS iterations after the learned warm start */
  double fallback_tau;   /* tower residual [m/s] above which the plain solve is redone */
  const double* mlp;     /* MLP parameters (layout OR_MLP_*), used when warm_start == 2 */
  int32_t friction_cone; /* 0: per-axis clip of Eq. (coulomb_pgs); 1: the tangent pair projected onto
                            the disc of radius mu lambda_n (the circular cone of the PGS figure) */
  int32_t restitution_bias;  /* 0: (1 + e) v_n in every iteration (Eq. (lambda_n) as printed); 1: the
                            normal row targets -e v_n- (pre-solve normal velocity) when the point
                            approaches faster than 2 |g| dt, else 0 */
  int32_t manifold_mode; /* 0: literal silhouettes clipped (Sec. "Contact Manifold (Face Clipping)");
                            1: reference-face clipping */
  int32_t mega_bodies;   /* towers of at least this many bodies (0: none) take the partitioned colouring */
  int32_t colour_partition;  /* bodies per colouring partition (tower-local index / this) */
  int32_t _pad;
} or_params;

/* Learned warm start: per-contact MLP 24 -> 128 -> 128 -> 3 with GELU (erf form).  Its outputs
 * are added to the previous step's dimensionless impulses (features 12..14) and the sum y maps to
 * lambda_n = max(0, y_n) |g| dt / k_n, lambda_t = clip(y_t |g| dt / k_t, +-mu lambda_n).  Parameters
 * as doubles (already rounded to bfloat16 by the caller) in this order:
 * W1[24][128], b1[128], W2[128][128], b2[128], W3[128][3], b3[3], mean[24], std[24].
 * Each layer's input is rounded to bfloat16, as the GPU feeds its matrix cores. */
#define OR_NFEAT 24
#define OR_HIDDEN 128
#define OR_MLP_SIZE (24 * 128 + 128 + 128 * 128 + 128 + 128 * 3 + 3 + 24 + 24)
/* Per-point record written when feature output is requested: 24 features, k[3], lambda[3]. */
#define OR_FEAT_RECORD 30

typedef struct {
  int32_t body;          /* tower-local body index */
  int32_t start;         /* first step on which the force acts */
  int32_t steps;         /* number of steps it acts */
  int32_t _pad;
  double force[3];       /* world-frame force at the centre of mass [N] */
  double withdraw;       /* displacement along the force that deactivates the body; 0 = never */
  double x0[3];          /* position at the start of the push (written by the oracle) */
} or_push;

/* One contact manifold (a colliding pair) with up to four points. */
typedef struct {
  int32_t a, b;          /* bodies; b = -1 is the ground (then the normal is -z) */
  int32_t colour, npts;
  int32_t axis;          /* SAT axis 0..14 (A0..A2, B0..B2, Ai x Bj row-major); -1 for ground */
  int32_t band;          /* precision-band flags (OR_BAND_*) */
  int32_t slot[4];       /* diagonal slot 0..3 (box pairs) or vertex index 0..7 (ground) */
  double normal[3], t1[3], t2[3];   /* normal points from a to b */
  double depth;          /* penetration used by the position correction */
  double sigma;          /* SAT separation -min_u delta_u (negative when overlapping) */
  double point[4][3];    /* world contact points */
  double lam[4][3];      /* accumulated impulses (normal, t1, t2) after the solve */
  double k[4][3];        /* inverse effective masses (normal, t1, t2) */
  double vbias[4];       /* restitution targets of the normal rows (restitution_bias) */
  double k12[4];         /* coupling of the two tangent rows (t1 and t2) of a point (disc friction) */
} or_manifold;

enum {
  OR_BAND_SEPARATION = 1,   /* |sigma| < 1e-6 m: the collide decision is precision sensitive */
  OR_BAND_NORMAL = 2,       /* two best non-parallel axes within 1e-6 m */
  OR_BAND_CROSS = 4,        /* a cross axis with |a x b| within 10% of the skip threshold */
  OR_BAND_CLIP = 8,         /* a slot extreme tied within 1e-6 m, or a merge within 10% of 1e-6 m */
  OR_BAND_GROUND = 16,      /* a vertex within 1e-6 m of the ground plane, or a depth tie at the cut */
  OR_BAND_EMPTY = 32        /* empty clip: the single support-midpoint fallback was used */
};

typedef struct {
  int64_t steps;
  int64_t candidates;      /* broadphase candidates, summed over steps */
  int64_t manifolds;       /* colliding pairs, summed over steps */
  int64_t points;          /* contact points, summed over steps */
  int64_t contact_iters;   /* points x iterations, summed over steps */
  int64_t fallbacks;       /* learned solves redone by the plain solver */
  int32_t colours;         /* colours used in the last step */
  int32_t error;           /* 1: colour cap exceeded (manifold dropped); 2: manifold capacity */
  double res_rms;          /* natural-map residual of the last solve, RMS over rows [m/s] */
  double res_max;          /* ... and max |r| */
} or_stats;

typedef struct {
  int32_t collide, axis, band, _pad;
  double depth, sigma;
  double normal[3];
} or_sat_result;

/* Eq. (rotmat): rotation matrix of a unit quaternion [w,x,y,z]; R row-major. */
void or_quat_to_rot(const double q[4], double R[9]);
/* Eq. (inertia): diagonal body inertia of a uniform box of mass m and half extents he. */
void or_box_inertia(double m, const double he[3], double I[3]);
/* Sec. "Narrowphase: OBB SAT": 15-axis test of boxes A and B. */
void or_sat(const double heA[3], const double xA[3], const double qA[4],
            const double heB[3], const double xB[3], const double qB[4], or_sat_result* out);
/* The same with the reference-face preference of the clipping variant: a colliding pair keeps its
 * best face axis unless a cross axis overlaps less than 0.95 of it minus 1e-6 m. */
void or_sat_ex(const double heA[3], const double xA[3], const double qA[4],
               const double heB[3], const double xB[3], const double qB[4], int32_t prefer_face,
               or_sat_result* out);
/* Sec. "Contact Manifold (Face Clipping)": manifold of a colliding box pair (normal from A to B). */
int or_manifold_box(const double heA[3], const double xA[3], const double qA[4],
                    const double heB[3], const double xB[3], const double qB[4],
                    const double normal[3], double depth, or_manifold* out);
/* The reference-face variant of the same (axis: the SAT axis 0..14 of the pair). */
int or_manifold_refface(const double heA[3], const double xA[3], const double qA[4],
                        const double heB[3], const double xB[3], const double qB[4],
                        const double normal[3], double depth, int axis, or_manifold* out);
/* Box against the ground half-space z <= 0; returns 1 if it collides. */
int or_manifold_ground(const double he[3], const double x[3], const double q[4], or_manifold* out);

/* Sec. "Contact Solver": PGS on explicit manifolds, processed in array order.
 * Bodies: inverse mass, world inverse inertia (row-major 3x3), position, velocities (updated).
 * Manifolds must have a, b, npts, normal, t1, t2, point set; lam holds the initial
 * impulses (already applied to v, w by the caller if nonzero) and receives the result.
 * Writes k.  Returns the residual (RMS and max) through res[2]. */
void or_pgs(int nb, const double* invm, const double* Iinv, const double* x, double* v, double* w,
            int nm, or_manifold* m, double mu, double restitution, int iters, double res[2]);
/* The same with the friction and restitution options of or_params (cone, bias). */
void or_pgs_ex(int nb, const double* invm, const double* Iinv, const double* x, double* v, double* w,
               int nm, or_manifold* m, double mu, double restitution, int cone, int bias, int iters,
               double res[2]);

/* Step one tower n_steps times (state arrays updated in place).
 * prev/nprev: previous step's manifolds for the warm start (may be NULL/0).
 * feat_out (may be NULL): OR_FEAT_RECORD doubles per contact point of the last substep, in
 * processing order (features before the solve, k and the solved impulses after it).
 * mout/mcap/nm_out: manifolds of the last substep, in colour-sorted processing order.
 * step_counter: global step number of the first step (incremented by n_steps). */
int or_step_tower(const or_params* p, int nb, const double* he, const double* mass,
                  double* x, double* q, double* v, double* w, uint8_t* active,
                  double mu, int npush, or_push* push, int64_t* step_counter, int n_steps,
                  const or_manifold* prev, int nprev,
                  or_manifold* mout, int mcap, int* nm_out, or_stats* st,
                  double* feat_out, int feat_cap, int* nfeat_out);

/* bfloat16 rounding (round to nearest even) of a double, returned as a double. */
double or_bf16(double x);
/* MLP forward of one feature vector (normalisation, three layers); y[3] out. */
void or_mlp_forward(const double* mlp, const double f[OR_NFEAT], double y[3]);

/* Broadphase candidates of one tower (pairs a<b, b = -1 ground), canonical order. */
int or_broadphase(int nb, const double* he, const double* mass, const double* x, const double* q,
                  const uint8_t* active, double margin, int32_t* pairs, int cap);

/* ---- episode criteria (Sec. "Stability Detection and Collapse"), episode_oracle.c ---- */
typedef struct {
  double fd;            /* f_d of Eq. (collapse): displacement over the block's length, 0.5 */
  double ek_collapse;   /* epsilon_k of Eq. (collapse), 5e-5 J */
  double theta_deg;     /* theta_th of Eq. (collapse), 30 degrees */
  double ek_rest;       /* rest threshold of simulate_until_rest, 1e-7 J */
  double eps;           /* support epsilon of Eq. (stability), 2 mm */
  int32_t rest_steps;   /* steps after the collapse at most, 400 */
  int32_t _pad;
} or_episode_params;

typedef struct {
  double ek;            /* kinetic energy of the active dynamic blocks [J] */
  double dx_max;        /* largest displacement from the episode's start [m] */
  double theta_max;     /* largest angle between a block's thickness axis and the vertical [rad] */
  double margin;        /* Eq. (stability) margin [m] (positive inside; -inf without a polygon) */
  double com[2];        /* horizontal centre of mass [m] */
  int32_t n_support;    /* support-polygon vertices */
  int32_t c_d, c_k, c_theta;   /* the three conditions of Eq. (collapse) */
} or_episode_metrics;

typedef struct {
  int32_t collapsed, done;          /* collapse declared; at rest (or out of steps) after it */
  int32_t collapse_step, rest_step; /* -1 = not reached */
  double imbalance;                 /* -margin at the end of the last step before the collapse [m] */
  or_episode_metrics last;          /* criteria at the end of the last step */
} or_episode_state;

/* Criteria of one tower's state; x0: positions at the episode's start. */
void or_episode_eval(const or_episode_params* E, int nb, const double* he, const double* mass,
                        const double* x, const double* q, const double* v, const double* w,
                        const uint8_t* active, const double* x0, or_episode_metrics* out);

/* One step of one tower under the episode rules (see episode_oracle.c); prev/mout as in
 * or_step_tower (manifolds of the previous and of this step). */
int or_step_episode(const or_params* p, const or_episode_params* E, int nb, const double* he, const double* mass,
                    double* x, double* q, double* v, double* w, uint8_t* active, double mu, int npush,
                    or_push* push, int64_t* step_counter, const double* x0, or_episode_state* es,
                    const or_manifold* prev, int nprev, or_manifold* mout, int mcap, int* nm_out, or_stats* st);

#ifdef __cplusplus
}
#endif
#endif
