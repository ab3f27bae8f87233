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
 *  - The world owns its device memory.  Host-side changes (bodies, pushes, friction,
 *    state, activity) are kept on the host until jg_commit, which sizes the packing,
 *    allocates or resizes device buffers and copies the changes over.  jg_step_batch
 *    then only queues kernel launches: it allocates no device memory, copies nothing
 *    and does not wait, and it refuses (JG_ESTATE) while host-side changes are not
 *    committed.
 *  - Every function returns a jg_status (0 = JG_OK, negative = error) and never
 *    throws.  jg_last_error() gives a thread-local message for the last error.
 *  - Calls on one world are not thread safe.  GPU work is queued on the stream
 *    given in jg_params.stream (NULL = the default stream); jg_step_batch returns
 *    without waiting; jg_sync and the jg_query_* calls wait for the stream
 *    ("syncing calls").
 *  - Device-side problems set bits of an error word (JG_ERR_*) and the step degrades
 *    deterministically: colliding pairs beyond a pack's capacity and manifolds beyond
 *    64 colours are dropped (the highest in canonical order first), and a tower whose
 *    state is non-finite at the start of a step is frozen (its bodies neither move nor
 *    collide and keep their state; the other towers step on, bit for bit as without it)
 *    until the host sets a new state.  The next syncing call does its work, then
 *    returns JG_ENAN (a non-finite state) or JG_ECAPACITY (a capacity bit) once for
 *    the bits raised since the previous syncing call; jg_query_stats keeps their OR.
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
  JG_ECAPACITY = -4,   /* a size limit was exceeded (the world's max_bodies, 65534 bodies per tower) */
  JG_ESTATE = -5,      /* call not valid in the world's current state */
  JG_ENAN = -6         /* a tower's state became non-finite */
} jg_status;

/* Device error-word bits reported by jg_query_stats. */
#define JG_ERR_CANDIDATES 1u   /* a body of an island in device memory had more than 16 broadphase candidates,
                                  or a tower stepped by the whole GPU exceeded its candidate capacity */
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
  int32_t warm_start;    /* 0: zero initial impulses; 1: previous step's impulses by key (same pair
                            and slot, normals within 0.95); 2: learned (network set by jg_set_mlp),
                            mlp_iters sweeps, plain re-solve of towers whose residual exceeds
                            fallback_tau */
  int32_t device;        /* HIP device ordinal */
  void* stream;          /* hipStream_t for all GPU work; NULL = default stream */
  int32_t pack_bodies;   /* bodies per on-chip pack (at most 256); 0 = automatic (one tower per pack when
                            the batch has no more towers than the GPU holds workgroups at once, else the
                            largest pack that keeps 8, or with features 4, workgroups per CU); -1 = every
                            tower keeps its state in device memory (the path of islands over 256 bodies) */
  float manifolds_per_body;  /* manifold capacity per body in a pack; 0 = automatic (3.5) */
  int32_t mlp_iters;     /* PGS iterations after a learned warm start; default 8 */
  double fallback_tau;   /* tower residual [m/s] above which a learned solve is redone plainly
                            (pre-solve velocities, zero impulses, iters sweeps); default 1e30 */
  int32_t record_features;   /* 1: keep per-point feature records of each launch's last step
                                (jg_query_features); default 0 */
  int32_t use_graph;     /* 1: jg_step_batch replays a HIP graph holding the launch (one graph per step
                            count, up to 8, built on first use and rebuilt when the layout, a device
                            buffer or a parameter changes), so that a loop of short calls pays one graph
                            launch per call; the results are those of the direct launch; default 0 */
  /* episode criteria (Sec. "Stability Detection and Collapse"; used after jg_begin_episodes) */
  double collapse_fd;    /* f_d of Eq. (collapse): a block moved more than f_d times its length; 0.5 */
  double collapse_ek;    /* epsilon_k of Eq. (collapse) [J]; 5e-5 */
  double collapse_theta; /* theta_th of Eq. (collapse) [degrees]; 30 */
  double rest_ek;        /* kinetic energy below which a collapsed tower is at rest [J]; 1e-7 */
  double support_eps;    /* eps of Eq. (stability): blocks whose lowest point is this close to the
                            ground support the tower [m]; 2e-3 */
  int32_t rest_steps;    /* steps after the collapse after which the tower is held even if not at
                            rest (Sec. "Full Floor Contact Simulation"); 400 */
  /* solver variants (Sec. "Contact Solver --- Projected Gauss-Seidel (PGS)") */
  int32_t friction_cone; /* 0: each tangent clipped to +-mu lambda_n (Eq. (coulomb_pgs)); 1: the two
                            tangent rows of a point solved from the same velocities with one inverse
                            effective mass (the larger eigenvalue of their 2 x 2 block) and their
                            impulse pair projected onto the disc of radius mu lambda_n (the circular
                            cone of the PGS figure); default 0 */
  int32_t restitution_bias;  /* 0: Eq. (lambda_n) as printed, (1 + e) times the current normal velocity
                            in every iteration; 1: the normal row drives the point's normal velocity to
                            -e v_n-, v_n- its normal velocity before any impulse of the step, when the
                            point approaches faster than 2 |g| dt (else to 0); default 0 */
  int32_t manifold_mode; /* 0: the literal silhouettes of Sec. "Contact Manifold (Face Clipping)"
                            (projected hulls of both boxes, one clipped by the other); 1: reference-face
                            clipping (the incident face clipped by the reference face's side planes,
                            points on or below the reference face, one point for an edge-edge axis);
                            default 0 */
  /* very large islands (Sec. "Discussion and Implications for Anastylosis": site-scale walls) */
  int32_t mega_bodies;   /* a tower of at least this many bodies is stepped by the whole GPU: one
                            cooperative launch whose phases span every CU, a uniform-grid broadphase
                            with no per-body candidate cap, 32-bit body indices (no 65,534-body
                            limit) and the partitioned colouring below; such towers take the zero
                            initial impulses (warm_start 0), no episode criteria, no feature records
                            and no graph replay; 0 = never; default 16384 */
  int32_t colour_partition;  /* bodies per colouring partition of such a tower: its pairs are coloured
                            greedily in four passes, each in canonical order: inside a partition (or
                            with the ground), between partitions p and p + 1 for even p, then for odd
                            p, then the rest; partitions of up to 2,048 bodies are walked in LDS; a
                            partition should span a course of a wall, so that a pair with the course
                            above joins the next partition; default 1024 */
  float mega_cand_per_body;  /* broadphase candidate capacity of such a tower, per body (the list is cut
                            at the first body whose candidates do not fit, JG_ERR_CANDIDATES); 16 */
  int32_t small_batch;   /* 0: a batch with at most two towers per CU, stepped with the zero or the
                            previous-step start and no feature records, gets one workgroup of four
                            waves per tower: the first steps it, all four build its manifolds, solve
                            it (each lane pair keeping one manifold's row terms in registers for the
                            whole solve) and sum its residual; the results are bit for bit those of
                            one wave per tower; -1: never; default 0 */
  int32_t precision;     /* arithmetic of the step kernels: JG_FP32 (the only one built; default).
                            JG_FP64 makes jg_create_world return JG_EINVAL: an FP64 instantiation
                            would double every kernel's LDS and registers, and is not built */
} jg_params;

#define JG_FP32 0
#define JG_FP64 1

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
  int64_t fallbacks;       /* learned solves redone plainly, summed over steps */
} jg_stats;

/* Fill *p with the defaults listed above. */
void jg_default_params(jg_params* p);

/* Create an empty world on p->device (the problem statement of Sec. "Physics Engine": many
 * independent towers, each a set of rigid boxes on the ground).  max_towers / max_bodies bound
 * what may be added; the body state arrays are allocated here.  *out receives the handle (NULL
 * on failure; JG_EINVAL for bad parameters, JG_EDEVICE / JG_ENOMEM for device failures). */
int32_t jg_create_world(const jg_params* p, int32_t max_towers, int32_t max_bodies, jg_world** out);

/* Release the world and its device memory (waits for queued work).  NULL is accepted. */
int32_t jg_destroy_world(jg_world* w);

/* Add n boxes to tower `tower` (0 <= tower < max_towers; towers are numbered
 * densely by first use).  Each box is a rigid body with the state (x, q, v, omega) of
 * Sec. "State of a Rigid Body"; its body-frame inertia follows from the mass and the full
 * sizes by Eq. (inertia).  half_extents: n x 3 body-frame half sizes (> 0);
 * mass: n (> 0, or 0 for a static box); pos: n x 3; quat: n x 4 (normalised by
 * the library); linvel, angvel: n x 3 or NULL (zero).  body_ids_out (n, may be
 * NULL) receives the global body ids, assigned densely in call order.  Host side only
 * (takes effect at jg_commit); JG_ECAPACITY beyond max_bodies, JG_EINVAL for bad values. */
int32_t jg_add_boxes(jg_world* w, int32_t tower, int32_t n, const double* half_extents, const double* mass,
                     const double* pos, const double* quat, const double* linvel, const double* angvel,
                     int32_t* body_ids_out);

/* Static friction coefficient mu_s of Eq. (coulomb) / Eq. (coulomb_pgs) for one
 * tower, or for every tower when tower = -1.  Default 0.4. */
int32_t jg_set_friction(jg_world* w, int32_t tower, double mu);

/* Move types of Tab. ziglar: the centre block and a side block pushed along its length
 * (no torque, F = 3 mu m g), a side block pushed across it (torque, F = 4 mu m g). */
#define JG_MOVE_NONE (-1)
#define JG_MOVE_CENTER_X 0
#define JG_MOVE_SIDE_Y 1
#define JG_MOVE_SIDE_X 2

/* Schedule a constant world-frame force at the centre of mass of `body`, acting on
 * steps [start_step, start_step + n_steps) (Ziglar pushes, Eqs. 4 and 8).  When
 * withdraw > 0 the body is deactivated (removed) once its displacement along the
 * force since start_step reaches withdraw metres.  move: the push's move type (JG_MOVE_*) for
 * the episode counts of jg_query_episode, or JG_MOVE_NONE.  In a tower whose collapse has been
 * declared (jg_begin_episodes) no push acts and no block is withdrawn any more.  Host side only. */
int32_t jg_set_push(jg_world* w, int32_t body, const double force[3], int32_t start_step, int32_t n_steps,
                    double withdraw, int32_t move);

/* Activate (1) or remove (0) a body, as in the block withdrawal of Sec. "Effect of the
 * Friction Coefficient"; inactive bodies neither move nor collide.  Host side only. */
int32_t jg_set_active(jg_world* w, int32_t body, int32_t active);

/* Make the host-side changes since the last commit resident on the device: recompute the
 * packing and (re)allocate per-pack buffers after towers or pushes were added, copy bodies,
 * state, friction and pushes, and forget the previous step's impulses after a state change.
 * Waits for the copies.  A world with no pending change returns at once. */
int32_t jg_commit(jg_world* w);

/* Queue n_steps steps of every tower on the world's stream: each step is the pipeline of
 * Secs. "Rigid-Body Foundations", "Physics Engine --- Collision Detection" and "Contact
 * Solver --- Projected Gauss-Seidel (PGS)" listed at the top of this file, run n_sub times
 * with dt / n_sub.  Kernel launches only (see the conventions above); JG_ESTATE while
 * host-side changes wait for jg_commit, or for warm_start 2 without a network. */
int32_t jg_step_batch(jg_world* w, int32_t n_steps);

/* Copy the state (x, q, v, omega; Sec. "State of a Rigid Body") of bodies
 * [first_body, first_body + n) to host arrays (any may be NULL).  Syncing call. */
int32_t jg_query_state(jg_world* w, int32_t first_body, int32_t n, double* pos, double* quat, double* linvel,
                       double* angvel);

/* Overwrite the state of bodies [first_body, first_body + n) (any array may be NULL = keep;
 * quaternions are normalised, a zero quaternion is JG_EINVAL).  Host side only: takes effect
 * at jg_commit, which also unfreezes every tower and forgets the previous step's impulses. */
int32_t jg_set_state(jg_world* w, int32_t first_body, int32_t n, const double* pos, const double* quat,
                     const double* linvel, const double* angvel);

/* Active flags of bodies [first_body, first_body + n) (withdrawn bodies are 0).  Syncing call. */
int32_t jg_query_active(jg_world* w, int32_t first_body, int32_t n, uint8_t* active);

/* Contact points (Sec. "Contact Manifold (Face Clipping)") of one tower's last solved step with
 * their impulses (Eq. (lambda_n), Eq. (coulomb_pgs)), in solve order.  Writes at most
 * `capacity` records to out and the total count to *n_out.  Syncing call. */
int32_t jg_query_contacts(jg_world* w, int32_t tower, jg_contact* out, int32_t capacity, int32_t* n_out);

/* Counters of one tower, or the sum over towers when tower = -1 (then colours is the
 * max, the residuals are the max over towers, error_word the OR).  The residual is the
 * natural-map residual of the PGS rows after the solve (the complementarity conditions of
 * Eq. (non_pen) and Eq. (coulomb_pgs)).  Syncing call. */
int32_t jg_query_stats(jg_world* w, int32_t tower, jg_stats* out);

/* Diagnostics: GPU cycles spent per phase of the step kernel since the last call, summed
 * over all workgroups, in this order: 0 load/store and push bookkeeping, 1 forces and frames,
 * 2 broadphase + narrowphase, 3 colouring, 4 manifolds, 5 PGS (with warm start), 6 contact
 * output and warm-start store, 7 residual, 8 integration, 9 position correction.  Writes
 * min(n, 10) counters (further entries 0) and resets them.  Waits. */
int32_t jg_query_phase_cycles(jg_world* w, uint64_t* cycles, int32_t n);

/* Per-point records of the last step of the last launch (needs record_features = 1), in the
 * order of jg_query_contacts: JG_FEAT_RECORD floats each, the 24 network features taken before
 * the solve (layout described with jg_set_mlp), then k_n, k_t1, k_t2 (Eq. (keff)) and the solved
 * impulses.  tower = -1 returns every tower's records, grouped by on-chip pack.  Writes at most
 * `capacity` records and the total count to *n_out.  Waits. */
int32_t jg_query_features(jg_world* w, int32_t tower, float* out, int32_t capacity, int32_t* n_out);

/* Network for warm_start = 2: host FP32 parameter vector (JG_MLP_PARAMS values, layout below).
 * The world keeps a device copy and its packed form; call again to replace it. */
int32_t jg_set_mlp(jg_world* w, const float* params);

/* Number of towers and bodies added so far (host side). */
int32_t jg_world_size(jg_world* w, int32_t* n_towers, int32_t* n_bodies);

/* Wait for all queued work of the world.  Syncing call. */
int32_t jg_sync(jg_world* w);

/* Zero-copy views of the device state for a caller that keeps tensors on the GPU (the state
 * (x, q, v, omega) of Sec. "State of a Rigid Body"): component-major FP32 arrays
 * x[3][stride], q[4][stride] (w, x, y, z), v[3][stride], angvel[3][stride] in the world's
 * internal body order (jg_body_slots maps body ids to it); stride = max_bodies.  The world
 * owns the memory; the pointers stay valid until the next jg_commit that rebuilds the packing
 * (after towers or pushes were added) or jg_destroy_world.  Between jg_commit and the next
 * host-side setter the device arrays are authoritative: the caller may read or write them
 * between launches (ordered on the world's stream), and every setter or query first reads them
 * back.  A setter makes the host copy authoritative until jg_commit, which then overwrites the
 * device arrays.  JG_ESTATE while host-side changes wait for jg_commit.  Any output may be NULL. */
int32_t jg_device_views(jg_world* w, void** x, void** q, void** v, void** angvel, int32_t* stride);

/* One tower's episode (Sec. "Stability Detection and Collapse"), as of the end of the last step. */
typedef struct {
  int32_t collapsed;       /* Eq. (collapse) held at the end of some step (then pushes stop) */
  int32_t done;            /* held after the collapse: at rest (ek < rest_ek) or rest_steps later */
  int32_t collapse_step;   /* step that declared the collapse, -1 = none */
  int32_t rest_step;       /* step the tower came to rest after it, -1 = not (yet) */
  int32_t rounds;          /* moves (pushes with a move type) started by the collapse step, or by the
                              last step if there was none */
  int32_t torque_moves;    /* of those, JG_MOVE_SIDE_X moves */
  int32_t removed;         /* of those, blocks withdrawn */
  int32_t support_vertices;   /* vertices of the support polygon of Eq. (stability) */
  float ek;                /* kinetic energy of the tower's active blocks [J] */
  float dx_max;            /* largest displacement of a block since jg_begin_episodes [m] */
  float theta_max;         /* largest angle between a block's thickness axis and the vertical [rad] */
  float margin;            /* Eq. (stability): smallest signed distance of the centre of mass to the
                              support polygon's edges, positive inside [m]; -inf without a polygon */
  float imbalance;         /* -margin at the end of the last step before the collapse (or of the last
                              step) [m]; NaN if the first step collapsed */
  float com[2];            /* horizontal centre of mass [m] */
  float _pad;
} jg_episode;

/* Start an episode in every tower: the current positions become the reference of the displacement
 * criterion, and no tower is collapsed.  From then on every step evaluates the criteria of
 * Eq. (collapse) and Eq. (stability) for each tower and applies the episode rules.  Needs a
 * committed world (JG_ESTATE otherwise); a later jg_commit that rebuilds the packing (after towers or
 * pushes were added) ends the episodes.  Allocates the episode state on first use; waits. */
int32_t jg_begin_episodes(jg_world* w);

/* The episode of one tower (JG_ESTATE without jg_begin_episodes).  Syncing call. */
int32_t jg_query_episode(jg_world* w, int32_t tower, jg_episode* out);

/* Internal slots of bodies [first_body, first_body + n) in the arrays of jg_device_views
 * (valid until the packing is rebuilt).  JG_ESTATE while added towers or pushes wait for
 * jg_commit. */
int32_t jg_body_slots(jg_world* w, int32_t first_body, int32_t n, int32_t* slots);

/* Message of the last failed call on this thread ("" if none). */
const char* jg_last_error(void);

/* ---------------------------------------------------------------------------------------------
 * Learned warm start: a per-contact network predicts each contact point's initial impulses
 * (normal, t1, t2) before the PGS sweeps of Sec. "Contact Solver --- Projected Gauss-Seidel".
 * The network is 24 features -> 128 -> GELU -> 128 -> GELU -> 3 on bfloat16 matrix-core
 * operands with FP32 accumulation.
 *
 * Parameters are one FP32 vector of JG_MLP_PARAMS values, in this order:
 *   W1[24][128], b1[128], W2[128][128], b2[128], W3[128][3], b3[3], mean[24], sd[24]
 * W[i][j] multiplies input i into output j; the first JG_MLP_TRAINABLE values are trained,
 * mean and sd z-score the features.  Every weight and bias is rounded to bfloat16 (nearest
 * even) when packed; layer inputs are rounded to bfloat16 before each product.
 *
 * Features of a contact point (in the contact frame F = (n, t1, t2) unless noted), at the
 * velocities before the solve: F (x_B - x_A) [3]; q_A^-1 q_B with w >= 0 [4]; world normal [3];
 * depth [1]; mu [1]; previous step's impulses of the same (pair, slot) in the outputs' units,
 * lambda_d k_d / (|g| dt) with this step's k, zero if new [3];
 * F r_A [3]; F r_B [3]; F (relative velocity of B with respect to A at the point) [3].  The
 * ground acts as a body at (x_A, y_A, 0) with the identity orientation.
 * Outputs y are the change of the dimensionless impulses lambda_d k_d / (|g| dt) (k_d of
 * Eq. (keff)) from the previous step's (features 12..14): with s = y + those features, the
 * initial impulses are lambda_n = max(0, s_n) |g| dt / k_n and
 * lambda_t = clip(s_t |g| dt / k_t, -mu lambda_n, mu lambda_n).  A zero network is therefore the
 * previous-step warm start (with the tangents clipped to the friction box).
 *
 * The jg_mlp_* calls take DEVICE pointers owned by the caller, queue work on `stream`
 * (NULL = default stream) and return without waiting.
 * ------------------------------------------------------------------------------------------- */
#define JG_MLP_PARAMS 20147
#define JG_MLP_TRAINABLE 20099
#define JG_MLP_FEATURES 24
#define JG_FEAT_RECORD 30      /* per contact point: 24 features, k[3], solved impulses[3] */

/* Size of the packed (bfloat16 operand layout) copy of the parameters. */
int32_t jg_mlp_packed_bytes(size_t* bytes);

/* Pack params (JG_MLP_PARAMS floats) into packed (jg_mlp_packed_bytes bytes, 16-byte aligned). */
int32_t jg_mlp_pack(const float* params, void* packed, void* stream);

/* Network outputs y (n x 3) for feature rows feats (n x 24), with packed parameters. */
int32_t jg_mlp_forward(const void* packed, const float* feats, int32_t n, float* y, void* stream);

/* Workspace needed by jg_mlp_grad for a batch of n rows. */
int32_t jg_mlp_grad_workspace_bytes(int32_t n, size_t* bytes);

/* Mean squared error over the n x 3 outputs against targets (n x 3), and its gradient with
 * respect to the JG_MLP_TRAINABLE trainable parameters (grad: JG_MLP_TRAINABLE floats; loss:
 * one float, may be NULL).  packed must hold jg_mlp_pack(params).  The forward pass is the one
 * jg_mlp_forward runs; the backward pass treats the bfloat16 roundings as the identity. */
int32_t jg_mlp_grad(const float* params, const void* packed, const float* feats, const float* targets, int32_t n,
                    float* grad, float* loss, void* workspace, size_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory (code under graph capture, tight serving or
 * training loops, harnesses that forbid hipMalloc): jg_mlp_grad with its workspace replaced by a
 * static device array of the library (the partial sums of at most 256 workgroups, 20.6 MB per
 * device, held until the process ends; every n >= 1 fits, a batch that would need more is
 * JG_ECAPACITY).  Same arguments, kernels and results as jg_mlp_grad; allocates nothing.  Calls
 * that overlap on one device share the array and race: order them on one stream. */
int32_t jg_mlp_grad_noalloc(const float* params, const void* packed, const float* feats, const float* targets,
                            int32_t n, float* grad, float* loss, void* stream);

/* One AdamW step (decoupled weight decay, bias-corrected moments; step counts from 1) on the
 * trainable parameters: p *= 1 - lr wd; m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
 * p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).  m, v: JG_MLP_TRAINABLE floats. */
int32_t jg_mlp_adamw(float* params, const float* grad, float* m, float* v, int32_t step, float lr, float beta1,
                     float beta2, float eps, float weight_decay, void* stream);

#ifdef __cplusplus
}
#endif
#endif
