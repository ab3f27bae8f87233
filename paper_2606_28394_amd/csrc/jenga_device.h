// Internal interface between the host library and the step kernel (gfx950).
//
// Device data layout (all FP32 unless noted), bodies in "internal order": the
// towers of pack 0, then pack 1, ...; the bodies of one tower are contiguous.
//   body SoA    x[3][cap], q[4][cap], v[3][cap], w[3][cap]         (component-major)
//   body static he[3][cap], mass[cap], flags[cap] (u32), tower[cap] (i32)
//   packs       pack_body0[np+1], pack_tower0[np+1], pack_push0[np+1]
//   towers      tower_body0[nt+1], tower_mu[nt]
//   pushes      body, start, steps (i32), force[3], withdraw, x0[3] per row (grouped by pack)
// A pack is the unit of one workgroup: its bodies, contacts and colours live in
// LDS for every step of a launch.
#pragma once
#include <stdint.h>

namespace jg {

constexpr uint32_t kActive = 1u;    // body takes part in the simulation
constexpr uint32_t kDynamic = 2u;   // mass > 0 (written by the solver)
constexpr int kMaxColours = 64;
constexpr int kWave = 64;

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
  const int32_t* tower_body0;
  const float* tower_mu;
  int32_t n_packs;
  // pushes
  const int32_t* push_body;
  const int32_t* push_start;
  const int32_t* push_steps;
  const float* push_force;     // [row][3]
  const float* push_withdraw;
  float* push_x0;              // [row][3]
  // per tower outputs (accumulated per launch, added by the host)
  uint32_t* tower_count;       // [tower][4]: candidates, manifolds, points, colours(last)
  float* tower_res;            // [tower][2]: rms, max of the last solve
  uint32_t* pack_error;        // [pack]
  // contacts of the last step (per pack, capacity pc manifolds)
  uint32_t* out_ab;            // [pack*pc + m]  a | b << 16 (pack-local, b = 0xffff ground)
  uint32_t* out_meta;          // npts | colour << 4 | slots << 12 (4 x 4 bits) | tower-in-pack << 28 unused
  float* out_geo;              // [pack*pc + m][8]: n[3], t1[3], depth, pad
  float* out_pts;              // [pack*pc + m][4][6]: point[3], lambda[3]
  int32_t* out_count;          // [pack]
  int32_t* out_tower;          // [pack*pc + m] pack-local tower index
  // previous-step impulses (warm start), canonical order per pack
  uint32_t* prev_key;          // [pack*pc + p]
  float* prev_data;            // [pack*pc + p][16]: n[3], slots(as bits), lambda[4][3]
  int32_t* prev_count;         // [pack]
  // parameters
  float g[3];
  float dt;                    // substep length
  float restitution, beta, slop, margin;
  int32_t iters, n_sub, n_steps, warm_start;
  int64_t step0;
  // pack capacities (LDS layout)
  int32_t nbp;     // bodies per pack
  int32_t pc;      // manifolds per pack
  int32_t cc;      // broadphase candidates per pack
  int32_t tpc;     // towers per pack
  int32_t ppc;     // push rows per pack
};

// LDS words needed by one pack with these capacities.
inline int64_t lds_words(int nbp, int pc, int cc, int tpc, int ppc, int warm) {
  int64_t w = 0;
  w += (int64_t)nbp * 42;           // body state, statics, frames, colour masks, tower idx
  w += (int64_t)tpc * 10;           // tower ranges, mu, counters, residual
  w += (int64_t)ppc * 10;           // push rows
  w += 2 * (kMaxColours + 1) + 16;  // colour offsets/counts, scalars
  w += cc;                          // candidates
  w += (int64_t)pc * 6;             // canonical pair list
  w += (int64_t)pc * 34;            // sorted manifolds and their points
  if (warm) w += (int64_t)pc * 17;  // previous step's impulses
  return w;
}

void launch_step(const StepArgs& a, int threads, size_t lds_bytes, void* stream);

}  // namespace jg
