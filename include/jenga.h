/*
 * jenga.h — C ABI of the MI355X (gfx950) batched block-stepping library.
 *
 * A world holds many independent towers ("islands") of oriented boxes, each
 * standing on its own static ground half-space z <= 0.  One call to
 * jg_step_batch advances every tower by n steps on the GPU, each step running
 * (Secs. "Rigid-Body Foundations", "Physics Engine --- Collision Detection",
 * "Contact Solver --- Projected Gauss-Seidel (PGS)" of the paper):
 *   external forces -> frames and AABBs -> broadphase (Eq. (aabb)) -> 15-axis SAT
 *   -> manifolds (projected hulls, clipped, <= 4 points) -> greedy colouring
 *   -> coloured PGS (Eq. (lambda_n), Eq. (coulomb_pgs)) -> residual
 *   -> semi-implicit integration (Eq. (quat_int), Eq. (newton_euler))
 *   -> Baumgarte correction (Eq. (baumgarte)).
 *
 * Conventions
 *  - SI units.  Quaternions are [w, x, y, z] (Sec. "State of a Rigid Body").
 *    Angular velocities are world-frame.  Body x is the box's length axis.
 *  - All host arrays are owned by the caller, row-major, double precision:
 *    vec3 arrays are n x 3, quaternion arrays n x 4.  The library copies them.
 *  - The world owns its device memory; it is allocated by jg_create_world and
 *    when towers are added, never inside jg_step_batch.
 *  - Every function returns a jg_status (0 = JG_OK, negative = error) and never
 *    throws.  jg_last_error() gives a thread-local message for the last error.
 *  - Calls on one world are not thread safe.  GPU work is queued on the stream
 *    given in jg_params.stream (NULL = the default stream); jg_step_batch returns
 *    without waiting, the jg_query_* calls wait for the stream.
 *  - Device-side problems (capacity overflow, colour cap, non-finite state) set
 *    an error word; the step drops the excess deterministically and the next
 *    jg_query_stats reports it.
 */
#ifndef JENGA_H
#define JENGA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct jg_world jg_world;

typedef enum {
  JG_OK = 0,
  JG_EINVAL = -1,      /* bad argument (null pointer, index or size out of range) */
  JG_ENOMEM = -2,      /* device or host allocation failed */
  JG_EDEVICE = -3,     /* a HIP call failed (message in jg_last_error) */
  JG_ECAPACITY = -4,   /* a tower does not fit the on-chip island capacity */
  JG_ESTATE = -5,      /* call not valid in the world's current state */
  JG_ENAN = -6         /* a tower's state became non-finite */
} jg_status;

/* Device error-word bits reported by jg_query_stats. */
#define JG_ERR_CANDIDATES 1u   /* reserved (broadphase candidates are consumed as produced) */
#define JG_ERR_MANIFOLDS 2u    /* colliding pairs exceeded the pack capacity */
#define JG_ERR_COLOURS 4u      /* a manifold needed more than 64 colours (dropped) */
#define JG_ERR_NAN 8u          /* non-finite body state */

typedef struct {
  double gravity[3];     /* m/s^2; default (0, 0, -9.81), Sec. "Equations of Motion" */
  double dt;             /* step length; default 1/240 s */
  double restitution;    /* e in Eq. (lambda_n); default 0.10 (appendix table) */
  double beta;           /* Baumgarte factor, Eq. (baumgarte); default 0.35 */
  double slop;           /* Baumgarte slop; default 4e-4 m */
  double margin;         /* AABB margin epsilon, Eq. (aabb); default 2e-3 m */
  int32_t n_sub;         /* substeps per step, each a full pipeline with dt/n_sub; default 1 */
  int32_t iters;         /* PGS iterations; default 20 */
  int32_t warm_start;    /* 0: zero initial impulses; 1: previous step's impulses by key */
  int32_t device;        /* HIP device ordinal */
  void* stream;          /* hipStream_t for all GPU work; NULL = default stream */
  int32_t pack_bodies;   /* bodies per on-chip pack; 0 = automatic */
  float manifolds_per_body;  /* manifold capacity per body in a pack; 0 = automatic (3.5) */
} jg_params;

/* One contact point of the last solved step. */
typedef struct {
  int32_t tower;         /* tower index */
  int32_t body_a;        /* body id (as returned by jg_add_boxes) */
  int32_t body_b;        /* body id, or -1 for the ground */
  int32_t slot;          /* diagonal slot 0..3 (box pair) or vertex 0..7 (ground) */
  int32_t colour;        /* PGS colour of the manifold */
  int32_t order;         /* position of the manifold in the tower's solve order */
  float point[3];        /* world contact point */
  float normal[3];       /* unit normal from body_a to body_b (-z for the ground) */
  float t1[3];           /* first tangent (the second is normal x t1) */
  float depth;           /* penetration of the manifold used by the position correction */
  float lambda_n, lambda_t1, lambda_t2;   /* accumulated impulses [N s] */
} jg_contact;

typedef struct {
  int64_t steps;           /* steps taken by this tower */
  int64_t candidates;      /* broadphase candidates, summed over steps */
  int64_t manifolds;       /* colliding pairs, summed over steps */
  int64_t points;          /* contact points, summed over steps */
  int64_t contact_iters;   /* points x PGS iterations, summed over steps */
  int32_t colours;         /* colours of the last step */
  uint32_t error_word;     /* JG_ERR_* bits */
  double residual_rms;     /* natural-map residual of the last solve, RMS over rows [m/s] */
  double residual_max;     /* largest |row residual| of the last solve [m/s] */
} jg_stats;

/* Fill *p with the defaults listed above. */
void jg_default_params(jg_params* p);

/* Create an empty world on p->device.  max_towers / max_bodies bound what may be
 * added.  *out receives the handle (NULL on failure). */
int32_t jg_create_world(const jg_params* p, int32_t max_towers, int32_t max_bodies, jg_world** out);

/* Release the world and its device memory (waits for queued work). */
int32_t jg_destroy_world(jg_world* w);

/* Add n boxes to tower `tower` (0 <= tower < max_towers; towers are numbered
 * densely by first use).  half_extents: n x 3 body-frame half sizes (> 0);
 * mass: n (> 0, or 0 for a static box); pos: n x 3; quat: n x 4 (normalised by
 * the library); linvel, angvel: n x 3 or NULL (zero).  body_ids_out (n, may be
 * NULL) receives the global body ids, assigned densely in call order. */
int32_t jg_add_boxes(jg_world* w, int32_t tower, int32_t n, const double* half_extents, const double* mass,
                     const double* pos, const double* quat, const double* linvel, const double* angvel,
                     int32_t* body_ids_out);

/* Static friction coefficient mu_s of Eq. (coulomb) / Eq. (coulomb_pgs) for one
 * tower, or for every tower when tower = -1.  Default 0.4. */
int32_t jg_set_friction(jg_world* w, int32_t tower, double mu);

/* Schedule a constant world-frame force at the centre of mass of `body`, acting on
 * steps [start_step, start_step + n_steps) (Ziglar pushes, Eqs. 4 and 8).  When
 * withdraw > 0 the body is deactivated (removed) once its displacement along the
 * force since start_step reaches withdraw metres. */
int32_t jg_set_push(jg_world* w, int32_t body, const double force[3], int32_t start_step, int32_t n_steps,
                    double withdraw);

/* Activate (1) or remove (0) a body; inactive bodies neither move nor collide. */
int32_t jg_set_active(jg_world* w, int32_t body, int32_t active);

/* Queue n_steps steps of every tower on the world's stream (one kernel launch).  Changes made
 * on the host since the last call (bodies, pushes, state, friction) are copied to the device
 * first; n_steps = 0 only does that copy.  The on-chip packing is recomputed (and per-pack
 * buffers reallocated) after towers or pushes were added. */
int32_t jg_step_batch(jg_world* w, int32_t n_steps);

/* Copy bodies [first_body, first_body + n) to host arrays (any may be NULL).  Waits. */
int32_t jg_query_state(jg_world* w, int32_t first_body, int32_t n, double* pos, double* quat, double* linvel,
                       double* angvel);

/* Overwrite bodies [first_body, first_body + n) (any array may be NULL = keep). */
int32_t jg_set_state(jg_world* w, int32_t first_body, int32_t n, const double* pos, const double* quat,
                     const double* linvel, const double* angvel);

/* Active flags of bodies [first_body, first_body + n).  Waits. */
int32_t jg_query_active(jg_world* w, int32_t first_body, int32_t n, uint8_t* active);

/* Contact points of one tower's last solved step, in solve order.  Writes at most
 * `capacity` records to out and the total count to *n_out.  Waits. */
int32_t jg_query_contacts(jg_world* w, int32_t tower, jg_contact* out, int32_t capacity, int32_t* n_out);

/* Counters of one tower, or the sum over towers when tower = -1 (then colours is the
 * max, the residuals are the max over towers, error_word the OR).  Waits. */
int32_t jg_query_stats(jg_world* w, int32_t tower, jg_stats* out);

/* Diagnostics: GPU cycles spent per phase of the step kernel since the last call, summed
 * over all workgroups, in this order: 0 load/store and push bookkeeping, 1 forces and frames,
 * 2 broadphase + narrowphase, 3 colouring, 4 manifolds, 5 PGS (with warm start), 6 contact
 * output and warm-start store, 7 residual, 8 integration, 9 position correction.  Writes
 * min(n, 10) counters (further entries 0) and resets them.  Waits. */
int32_t jg_query_phase_cycles(jg_world* w, uint64_t* cycles, int32_t n);

/* Number of towers and bodies added so far. */
int32_t jg_world_size(jg_world* w, int32_t* n_towers, int32_t* n_bodies);

/* Wait for all queued work of the world. */
int32_t jg_sync(jg_world* w);

/* Message of the last failed call on this thread ("" if none). */
const char* jg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
