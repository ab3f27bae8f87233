// Internal interface between the host library and the step kernel (gfx950).
//
// Device data layout (all FP32 unless noted), bodies in "internal order": the
// towers of pack 0, then pack 1, ...; the bodies of one tower are contiguous.
//   body SoA    x[3][cap], q[4][cap], v[3][cap], w[3][cap]         (component-major)
//   body static he[3][cap], mass[cap], flags[cap] (u32), tower[cap] (i32)
//   packs       pack_body0[np+1], pack_tower0[np+1], pack_push0[np+1], pack_slot0[np+1]
//   towers      tower_body0[nt+1], tower_mu[nt]
//   pushes      body, start, steps (i32), force[3], withdraw, x0[3] per row (grouped by pack)
//   contacts    per pack, slots [pack_slot0[p], pack_slot0[p+1]) of the output / warm-start arrays
// A pack is the unit of one workgroup: its bodies, contacts and colours live in
// LDS for every step of a launch.  Packs are launched in size classes, each with
// the LDS its largest pack needs.  An island too large for LDS (more than 256 bodies) is a
// "global" pack: the same layout lives in a per-pack region of device memory instead.
#pragma once
#include <stdint.h>

#include <string>

namespace jg {

constexpr uint32_t kActive = 1u;    // body takes part in the simulation
constexpr uint32_t kDynamic = 2u;   // mass > 0 (written by the solver)
constexpr uint32_t kHeld = 4u;      // on chip only: an active body of a frozen tower (treated as
                                    // inactive; written back as active)
constexpr int kMaxColours = 64;
constexpr int kWave = 64;
constexpr int kRing = 128;          // broadphase -> narrowphase candidate ring
// phases timed by the step kernel: load/store, forces+frames, broad+narrow, colouring,
// manifolds, PGS (with warm start), outputs, residual, integration, position correction
constexpr int kPhases = 10;

struct StepArgs {
  // bodies
  float* x;
  float* q;
  float* v;
  float* w;
  const float* he;
  const float* mass;        // 0 = static
  uint32_t* flags;
  const int32_t* body_tower;
  int32_t cap;              // body array stride
  // packs / towers
  const int32_t* pack_body0;
  const int32_t* pack_tower0;
  const int32_t* pack_push0;
  const int32_t* pack_slot0;
  const int64_t* pack_goff;    // [pack] word offset of the pack's region in gmem
  float* gmem;                 // per-pack regions: the contact points' lever arms and impulses
                               // (kManDevWords per manifold slot), their restitution targets
                               // (kManBiasWords per slot), the narrowphase's normals and
                               // depths (kManSatWords per slot), then, for a pack whose layout
                               // lives in device memory, the whole layout
  int32_t in_gmem;             // 1: this launch's packs keep their whole layout in gmem
  int32_t hot_bodies;          // in_gmem packs: 1 = the arrays of the serial walks also in LDS
  const int32_t* tower_body0;
  const float* tower_mu;
  int32_t pack_first;          // first pack of this launch
  int32_t n_packs;             // packs in this launch
  // pushes
  const int32_t* push_body;
  const int32_t* push_start;
  const int32_t* push_steps;
  const float* push_force;     // [row][3]
  const float* push_withdraw;
  float* push_x0;              // [row][3]
  // per tower outputs (accumulated per launch, folded in by the host)
  uint32_t* tower_count;       // [tower][4]: candidates, manifolds, points, colours(last)
  float* tower_res;            // [tower][2]: rms, max of the last solve
  uint32_t* pack_error;        // [pack]
  uint32_t* err_flag;          // one word: error bits raised since the host last read it
  uint32_t* tower_frozen;      // [tower] 1 = the tower's state was found non-finite: it is held
  // episodes (Sec. "Stability Detection and Collapse"); ep_state null = not tracked
  uint32_t* ep_state;          // [tower][kEpisodeWords] (see kEp*)
  const float* ep_x0;          // [3][cap] positions at the episode's start
  float ep_fd, ep_ek_collapse, ep_cos_theta, ep_ek_rest, ep_eps;
  int32_t ep_rest_steps;
  // contacts of the last step
  uint32_t* out_ab;            // [slot]  a << 16 | b (pack-local, b = 0xffff ground)
  uint32_t* out_meta;          // npts | colour << 4 | slots << 12 (4 x 4 bits)
  float* out_geo;              // [slot][8]: n[3], t1[3], depth, pad
  float* out_pts;              // [slot][4][6]: point[3], lambda[3]
  int32_t* out_count;          // [pack]
  int32_t* out_tower;          // [slot] pack-local tower index
  // previous-step impulses (warm start), canonical order per pack
  uint32_t* prev_key;          // [slot]
  float* prev_data;            // [slot][16]: n[3], slots(as bits), lambda[4][3]
  int32_t* prev_count;         // [pack]
  // cycles spent per phase, summed over packs (kPhases counters)
  unsigned long long* phase_cycles;
  // learned warm start (warm_start == 2) and per-point feature records
  const void* mlp;             // packed network (16-byte aligned, jg_mlp_pack layout)
  float* feat_out;             // [slot][4][30]: features, k, impulses of the last step; or null
  uint32_t* tower_fallback;    // [tower][2]: fallbacks, fallback points (accumulated per launch)
  int32_t mlp_iters;
  float fallback_tau;
  // parameters
  float g[3];
  float dt;                    // substep length
  float restitution, beta, slop, margin;
  int32_t iters, n_sub, n_steps, warm_start;
  int32_t friction_cone;       // 1: tangent pairs projected onto the disc of radius mu lambda_n
  int32_t restitution_bias;    // 1: normal rows target -e v_n- (pre-solve velocity) above 2 |g| dt
  int32_t manifold_mode;       // 0: literal silhouettes; 1: reference-face clipping
  int64_t step0;
  // capacities of this launch (LDS layout)
  int32_t lat;     // 1: one tower per 256-thread workgroup (small batches), sweeps from registers
  int32_t nbp;     // bodies per pack
  int32_t pc;      // manifolds per pack
  int32_t tpc;     // towers per pack
  int32_t ppc;     // push rows per pack
};

constexpr int kBodyWords = 28;     // x3 q4 v3 w3 he3 invm flag tower Iw6 aabb/mask3
constexpr int kTowerWords = 14;    // body range, mu, counters4, residual2, canonical range2, points, frozen
constexpr int kPushWords = 10;
constexpr int kManWords = 4;       // canonical (code, pos) + sorted (code, meta)
constexpr int kManDevWords = 28;   // r_A 12, lambda 12, n 3, depth per sorted manifold, in the
                                   // pack's device region
constexpr int kManBiasWords = 4;   // restitution targets of a sorted manifold's points (after all
                                   // of the pack's records; used with restitution_bias only)
constexpr int kManSatWords = 4;    // the narrowphase's normal and depth of a canonical colliding
                                   // pair (after the targets), reused to build its manifold
constexpr int kManPackWords = kManDevWords + kManBiasWords + kManSatWords;   // per slot of a pack
constexpr int kWarmWords = 18;     // sorted -> canonical map + previous step store (17)
constexpr int kStageWords = 64 * 16 + 64 * 3;   // network input rows of one 64-point chunk (bf16)
constexpr int kLearnedIslandWaves = 4;          // waves of a pack in device memory with the network
                                                // and the chunk's previous dimensionless impulses
constexpr int kFeatRecord = 30;

// per-tower episode words: flags (kEpCollapsed | kEpDone), collapse step, rest step (-1 = not
// reached), support-polygon vertices, then floats: kinetic energy, largest displacement, largest
// tilt, margin of Eq. (stability) at the end of the last step, imbalance (-margin one step before
// the collapse), centre of mass x, y
constexpr int kEpisodeWords = 12;
constexpr uint32_t kEpCollapsed = 1u, kEpDone = 2u;
enum { kEpFlags = 0, kEpCollapseStep, kEpRestStep, kEpSupport, kEpEk, kEpDx, kEpTheta, kEpMargin, kEpImbalance,
       kEpComX, kEpComY };

constexpr int kRegBodies = 256;    // largest pack the LDS path takes (register broadphase windows)

// words of the window bounding boxes a global pack's broadphase keeps (6 per 64 bodies)
__host__ __device__ inline int64_t window_words(int nbp) { return 6 * (int64_t)((nbp + 63) / 64); }

// an island in device memory lists its broadphase candidates of a step: at most this many per
// body (more sets JG_ERR_CANDIDATES and keeps the first ones)
constexpr int kCandPerBody = 16;

// LDS words of a pack kept in device memory: its small arrays (phase counters, colour offsets,
// the candidate ring, towers, pushes, broadphase windows) and, with `bodies`, the body arrays
// that the serial walks (broadphase, colouring) read: positions, AABB half sizes and colour
// masks, flags, colouring lane masks (9 words per body)
constexpr int kHotBodyWords = 9;
__host__ __device__ inline int64_t hot_words(int nbp, int tpc, int ppc, bool bodies) {
  int64_t w = 2 * kPhases + 2 * (kMaxColours + 1) + 16 + kRing + (int64_t)tpc * kTowerWords +
              (int64_t)ppc * kPushWords + window_words(nbp);
  if (bodies) w += (int64_t)kHotBodyWords * nbp;
  return w;
}

// LDS layout modes: 0 plain; 1 previous-step store (warm start from the previous step, or
// feature records); 2 learned warm start: the store plus network input staging, saved
// velocities (6 per body), residual partials (2 per manifold), fallback state (3 per tower).
inline int64_t lds_words(int nbp, int pc, int tpc, int ppc, int mode) {
  int64_t w = 0;
  w += (int64_t)nbp * kBodyWords;
  w += (int64_t)tpc * kTowerWords;
  w += (int64_t)ppc * kPushWords;
  w += 2 * (kMaxColours + 1) + 16 + kRing + 2 * kPhases;
  w += (int64_t)pc * kManWords;
  if (mode >= 1) w += (int64_t)pc * kWarmWords;
  if (mode == 2) w += kStageWords + 6 * (int64_t)nbp + 2 * (int64_t)pc + 3 * (int64_t)tpc;
  return w;
}

// queues one launch of the step kernel; returns the hipError_t of the launch (0 = success)
int launch_step(const StepArgs& a, size_t lds_bytes, void* stream);

// the kernel variant and workgroup size launch_step uses for these arguments (one workgroup
// per pack, dynamic LDS as given to launch_step), for a kernel node of a graph; sets the
// variants' dynamic-LDS limit on the current device first; returns a hipError_t (0 = success)
int step_launch_config(const StepArgs& a, const void** func, unsigned* block_threads);

// records the message returned by jg_last_error on this thread; returns code
int32_t set_error(int32_t code, const std::string& msg);

// ------------------------------------------------------------------------------------------------
// Islands stepped by the whole GPU (towers of at least mega_bodies bodies): one cooperative launch
// of every step, its phases separated by grid-wide barriers, 32-bit body indices.  The island's
// bodies are the internal range [g0, g0 + nb) of the world arrays; its pushes the rows [p0, p0 + np)
// (push_body holds internal indices).  Scratch arrays are sized by the host from nb and cand_cap.
// ------------------------------------------------------------------------------------------------
constexpr int kMegaThreads = 256;
constexpr int kMegaBodyWords = 26;   // x3 q4 v3 w3 he3 invm Iw6 hm3 (SoA, stride nb)
constexpr int kMegaBodyU32 = 8;      // flag, tower (0), colour mask lo, hi, cell, candidate count,
                                     // candidate offset, cell-sorted body (stride nb)
constexpr int kMegaScal = 256;       // scalar words (counters, colour tables)
constexpr int kMegaStagedPartition = 2048;  // colouring partitions up to this size are walked in LDS
constexpr int kMegaChunk = 1024;            // pairs staged in LDS per walk chunk

struct MegaArgs {
  float *x, *q, *v, *w;
  const float *he, *mass;
  uint32_t* flags;
  int32_t cap, g0, nb;
  int32_t tslot;               // tower slot (statistics, frozen flag)
  float mu;
  const int32_t *push_body, *push_start, *push_steps;
  const float *push_force, *push_withdraw;
  float* push_x0;
  int32_t p0, np;
  uint32_t* tower_count;       // [4 * tslot + k]: candidates, manifolds, points (added), colours (last)
  float* tower_res;            // [2 * tslot + k]: residual RMS, max (last substep)
  uint32_t* tower_frozen;
  uint32_t* err_flag;          // the world's error word (reported by the next syncing call)
  uint32_t* island_err;        // this island's error bits since the host last read them
  float g[3], dt, restitution, beta, slop, margin;
  int32_t iters, n_sub, n_steps, friction_cone, restitution_bias, manifold_mode, partition;
  int64_t step0;
  // scratch
  float* body;                 // kMegaBodyWords * nb
  uint32_t* ubody;             // kMegaBodyU32 * nb
  int32_t* cells;              // 2 * (ncell_cap + 1): counts, starts
  int32_t ncell_cap;
  uint32_t* cand;              // 3 * cand_cap: body a, body b (~0u: the ground), collide flag / position
  int32_t cand_cap;
  int32_t* man;                // 7 * cand_cap: canonical a, b, colour, sorted slot; sorted a, b, meta
  float* md;                   // kManDevWords * cand_cap, colour-sorted records
  float* mtb;                  // kManBiasWords * cand_cap, their restitution targets
  int32_t* part;               // nparts + 1 first canonical manifold of each partition, then nparts far counts
  int32_t nparts;
  float* red;                  // 2 * gridDim partial sums (residual)
  int32_t* ired;               // 2 * gridDim integer partials (scans, counts)
  int32_t* scal;               // kMegaScal words
  // contacts of the launch's last step, canonical order (npts 0: a pair dropped by the colouring)
  int32_t *out_a, *out_b;
  uint32_t* out_meta;          // npts | colour << 4 | slots << 12
  float *out_geo, *out_pts;    // 8 and 24 words per pair, as the packs' outputs
  int32_t* out_count;
};

// queues the cooperative launch of an island's steps (blocks from mega_blocks); a hipError_t
int launch_mega(const MegaArgs& a, int blocks, void* stream);
// the workgroups of the grid-wide kernel for an island of `bodies` bodies: every one resident at
// once (at most the occupancy of the current device times its CUs, two per CU); a hipError_t
int mega_blocks(int bodies, int* blocks);

}  // namespace jg
